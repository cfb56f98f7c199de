// The learned surrogate's network: MLP 32 -> 128 -> 128 -> 1 with GELU
// (erf form), bf16 operands on the matrix cores with fp32 accumulation, fp32
// master weights and Adam (Kingma & Ba, 2015).  It predicts y_i = c_ii
// (C^-1)_ii from the 32 local features of row i.
//
// Kernels
//   k_mlp_train   : one training step's gradient, fused: a persistent
//                   workgroup per compute unit (eight waves, 16 rows each per
//                   128-row tile) runs the forward layers, the weighted-MSE
//                   gradient back through layer 3 (fp32), layer 2 (dgrad) and
//                   both GELUs, and accumulates dW1 = Xn^T dz1 and dW2 =
//                   h1^T dz2 over its tiles in registers (the tiles' operands
//                   pass through LDS); bias, w3, b3 and loss sums per wave.
//                   Products on v_mfma_f32_16x16x32_bf16 (bf16 operands, fp32
//                   accumulation); the step's rows are drawn from Philox
//                   inside the kernel.  One partial row per workgroup.
//   k_mlp_forward : predictions, one 128-row tile per workgroup.
//   k_mlp_update  : gradient assembly (the partial rows summed in a fixed
//                   order), Adam step, bf16 copies of the weights.
// Rounding points (what the oracle reproduces): the normalised features,
// W1, W2, h1, dz2 and dz1 enter MFMA products as bf16 (nearest even); h2,
// w3, the biases and every elementwise step stay fp32.  GELU and its
// derivative use an erf approximation with absolute error at most 1.5e-7
// (gelu_terms), far below the bf16 rounding that follows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mcinv.h"
#include "boundary.h"
#include "surrogate_internal.h"
#include "device_common.h"
#include "mfma_tile.h"

namespace mcinv {

constexpr int kF = 32, kH = 128;
constexpr int oW1 = 0, ob1 = kF * kH, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, ow3 = ob2 + kH, ob3 = ow3 + kH;
constexpr int kParams = ob3 + 1;     // 20865
constexpr int kPart = 3 * kH + 2;    // db1, db2, dw3, db3, loss
constexpr int kWRow = ob2 + kPart;   // one weight-gradient partial row: W1 | b1 gap | W2 | block sums

typedef unsigned short bf16_t;

// round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ inline bf16_t to_bf16(float x) { return __builtin_bit_cast(bf16_t, (__bf16)x); }

struct MlpArgs {
    const float* X;          // raw features [N][32]
    const float* y;          // labels [N]
    const float* w;          // row weights [N]
    const int64_t* idx;      // rows of this call, or null: rows row0 + r
    int64_t row0;
    int32_t draw;            // nonzero: rows drawn from Philox (key, step) over N rows
    uint32_t key0, key1, step;
    int64_t N;
    int32_t R;               // rows of this call
    const float* mean;       // feature normalisation: (x - mean) * inv_std
    const float* inv_std;
    const bf16_t* W1T;       // [128][32]
    const bf16_t* W2T;       // [128 out][128 in]
    const bf16_t* W2;        // [128 in][128 out]
    const float* P;          // fp32 master parameters (biases, w3 read here)
    float* out;              // predictions [R]
    float* wpart;            // training: one partial row [kWRow] per workgroup
    float inv_denom;         // loss = sum_r w_r (out_r - y_r)^2 * inv_denom
};

// GELU (erf form) and its derivative at z: h = z Phi(z) and gp = Phi(z) +
// z phi(z), with Phi(z) = (1 + erf(z / sqrt 2)) / 2 and phi(z) = exp(-z^2 / 2)
// / sqrt(2 pi).
template <bool GP>
__device__ inline void gelu_terms(float z, float& h, float& gp)
{
    // GELU(z) = z Phi(z) with 2 Phi(z) = 1 + erf(z / sqrt 2), and
    // GELU'(z) = Phi(z) + z phi(z).  erfc(|x|) = (a1 t + ... + a5 t^5) e^{-x^2},
    // t = 1 / (1 + p |x|): Abramowitz & Stegun 7.1.26 (absolute error of erf
    // at most 1.5e-7).  With x = z / sqrt 2, e^{-x^2} = e^{-z^2/2} also gives
    // phi, so one hardware exp2 and one reciprocal serve both terms; for z < 0
    // the small tail Phi(z) = erfc(|x|) / 2 is formed without cancellation.
    constexpr float kRs2 = 0.70710678118654752f, kRs2pi = 0.39894228040143268f;
    constexpr float kHalfLog2e = 0.72134752044448170f;   // log2(e) / 2
    // the coefficients halved (exact), so that the product is Phi's tail
    constexpr float kP = 0.3275911f, kA1 = 0.5f * 0.254829592f, kA2 = 0.5f * -0.284496736f,
                    kA3 = 0.5f * 1.421413741f, kA4 = 0.5f * -1.453152027f, kA5 = 0.5f * 1.061405429f;
    const float t = __builtin_amdgcn_rcpf(fmaf(kP * kRs2, fabsf(z), 1.0f));
    const float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, kA5, kA4), kA3), kA2), kA1);
    const float g = __builtin_amdgcn_exp2f(-kHalfLog2e * z * z);   // e^{-z^2/2}
    const float q = poly * g;                                      // erfc(|z| / sqrt 2) / 2
    const float cdf = z < 0.0f ? q : 1.0f - q;                     // Phi(z)
    h = z * cdf;
    gp = GP ? fmaf(z * kRs2pi, g, cdf) : 0.0f;
}

// Row of the training data for step row r: the caller's list, a contiguous
// range, or the Philox draw floor(x N / 2^64) of the step (counter (r, step,
// 0x5EED, 0xA11CE), x = (o0 << 32) | o1).
__device__ inline int64_t mlp_row(const MlpArgs& a, int64_t r)
{
    if (a.draw) {
        uint32_t c0 = (uint32_t)r, c1 = a.step, c2 = 0x5EEDu, c3 = 0xA11CEu;
        Philox::block(c0, c1, c2, c3, a.key0, a.key1);
        const uint64_t x = ((uint64_t)c0 << 32) | c1;
        return (int64_t)(((unsigned __int128)x * (uint64_t)a.N) >> 64);
    }
    return a.idx ? a.idx[r] : a.row0 + r;
}

// Shared pieces of the forward and training kernels.
//
// Every product is taken transposed (hidden units on the M side of
// v_mfma_f32_16x16x32_bf16, a wave's 16 rows on N), so a product's result
// fragment -- lane (row r, group g) holding units 16t + 4g + v of row r -- is
// the next product's B operand as it stands: in the K step of 32 units
// covering tiles 2c and 2c + 1, lane group g holds units 32c + 4g .. 4g + 3
// and 32c + 16 + 4g .. + 3.  The weight rows in LDS carry their K units in
// that order (the 4-unit block b of a K step at position frag_block(b)).
//
// LDS arrays of 128 bf16 per row keep 16-byte chunk c of row r at chunk
// c ^ (r & 15), so that the 16 rows one fragment access touches fall in
// different banks; W1^T (32 per row) keeps chunk c at c ^ ((r >> 2) & 3).
constexpr int kMlpWaves = 8;
constexpr int kMlpRows = 16 * kMlpWaves;   // rows per tile (one workgroup)
// small vectors in LDS: feature mean and 1/std, b1, b2, w3, b3
constexpr int pMean = 0, pInv = kF, pB1 = 2 * kF, pB2 = pB1 + kH, pW3 = pB2 + kH, pB3 = pW3 + kH;
constexpr int kPb = pB3 + 1;
constexpr int kPartLd = (kPart + 3) / 4 * 4;

__device__ inline int frag_block(int b) { return b < 4 ? 2 * b : 2 * (b - 4) + 1; }

template <typename T>
__device__ inline T* sw128(T* base, int r, int col)
{
    return base + r * kH + ((((col >> 3) ^ (r & 15)) << 3) | (col & 7));
}
template <typename T>
__device__ inline T* sw32(T* base, int r, int col)
{
    return base + r * kF + ((((col >> 3) ^ ((r >> 2) & 3)) << 3) | (col & 7));
}

__device__ inline bf16x8 lds_bf16x8(const bf16_t* p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// two values to bf16 (nearest even) in one register, lo first
__device__ inline uint32_t pack_bf16(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t{lo, hi}), bf16x2_t));
}

template <int CTRL>
__device__ inline uint32_t dpp_u32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ inline float dpp_f32(float x)
{
    return __builtin_bit_cast(float, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, x)));
}

// Sums over the 16 lanes of a row of four values x[0..3] at once: lane b of
// each quad (b = lane & 3) gets the total of x[b].  Within the quad each lane
// hands two values to lane b ^ 2 and keeps the pair sums of x[2 (b >> 1)],
// x[2 (b >> 1) + 1], then one to lane b ^ 1; the quads' sums are then added
// across the row (row_ror 8, then row_ror 4, so that every lane of the row
// with the same b ends with the same bits: both steps pair commutatively).
__device__ inline float row16_sum4(float x0, float x1, float x2, float x3, int b)
{
    const bool hi = (b & 2) != 0, odd = (b & 1) != 0;
    const float y0 = (hi ? x2 : x0) + dpp_f32<0x4E>(hi ? x0 : x2);   // quad_perm [2, 3, 0, 1]
    const float y1 = (hi ? x3 : x1) + dpp_f32<0x4E>(hi ? x1 : x3);
    const float z = (odd ? y1 : y0) + dpp_f32<0xB1>(odd ? y0 : y1);   // quad_perm [1, 0, 3, 2]
    const float t = z + dpp_f32<0x128>(z);                            // row_ror 8
    return t + dpp_f32<0x124>(t);                                     // row_ror 4
}

// 4 x 4 transpose within a quad of lanes: lane b holds, for its row, units
// 0..3 as bf16 pairs (p01, p23); afterwards it holds unit b of the quad's rows
// 0..3 as (q01, q23).  The pairs first cross between lanes b and b ^ 2 (two
// units of two rows each), then single values between b and b ^ 1.
__device__ inline void quad_transpose(uint32_t p01, uint32_t p23, int b, uint32_t& q01, uint32_t& q23)
{
    const bool hi = (b & 2) != 0;
    const uint32_t y = dpp_u32<0x4E>(hi ? p01 : p23);
    const uint32_t A = hi ? y : p01, B = hi ? p23 : y;
    const uint32_t Ap = dpp_u32<0xB1>(A), Bp = dpp_u32<0xB1>(B);
    const uint32_t sel = (b & 1) ? 0x03020706u : 0x05040100u;
    q01 = __builtin_amdgcn_perm(Ap, A, sel);
    q23 = __builtin_amdgcn_perm(Bp, B, sel);
}

// The lane's four units (bf16 pairs p) of its row into a swizzled [unit][128
// rows] LDS array: after the quad transpose, unit urow (the caller's unit of
// quad lane b) of rows rcol .. rcol + 3 as one 8-byte write.
__device__ inline void put_transposed(bf16_t* base, int urow, int rcol, uint32_t p01, uint32_t p23, int b)
{
    uint32_t q01, q23;
    quad_transpose(p01, p23, b, q01, q23);
    *reinterpret_cast<uint2*>(sw128(base, urow, rcol)) = make_uint2(q01, q23);
}

// W1^T, W2^T (forward) and, for training, W2 (dgrad) from their global bf16
// copies into LDS (swizzled, K units in fragment order), with the small
// vectors.
template <bool TRAIN>
__device__ inline void stage_weights(const MlpArgs& a, bf16_t* w1t, bf16_t* w2p, bf16_t* w2q, float* pb)
{
    for (int t = threadIdx.x; t < kH * (kF / 8); t += blockDim.x) {
        const int r = t >> 2, c = t & 3;
        *reinterpret_cast<uint4*>(sw32(w1t, r, 8 * c)) = *reinterpret_cast<const uint4*>(a.W1T + r * kF + 8 * c);
    }
    for (int t = threadIdx.x; t < kH * (kH / 8); t += blockDim.x) {
        const int r = t >> 4, c8 = t & 15;
        const int col0 = 32 * (c8 >> 2), b = 2 * (c8 & 3);
        const uint4 g = *reinterpret_cast<const uint4*>(a.W2T + r * kH + 8 * c8);
        *reinterpret_cast<uint2*>(sw128(w2p, r, col0 + 4 * frag_block(b))) = make_uint2(g.x, g.y);
        *reinterpret_cast<uint2*>(sw128(w2p, r, col0 + 4 * frag_block(b + 1))) = make_uint2(g.z, g.w);
        if (TRAIN) {
            const uint4 h = *reinterpret_cast<const uint4*>(a.W2 + r * kH + 8 * c8);
            *reinterpret_cast<uint2*>(sw128(w2q, r, col0 + 4 * frag_block(b))) = make_uint2(h.x, h.y);
            *reinterpret_cast<uint2*>(sw128(w2q, r, col0 + 4 * frag_block(b + 1))) = make_uint2(h.z, h.w);
        }
    }
    for (int t = threadIdx.x; t < kPb; t += blockDim.x) {
        float v;
        if (t < pInv)
            v = a.mean[t - pMean];
        else if (t < pB1)
            v = a.inv_std[t - pInv];
        else if (t < pB2)
            v = a.P[ob1 + t - pB1];
        else if (t < pW3)
            v = a.P[ob2 + t - pB2];
        else if (t < pB3)
            v = a.P[ow3 + t - pW3];
        else
            v = a.P[ob3];
        pb[t] = v;
    }
}

// One data row of the call: the lane's eight features (group kg), label and
// weight.  The loads do not depend on whether the row exists (a row past the
// end loads row R - 1 of the call and is flagged), so that nothing waits for
// them before their first use.
struct RowIn {
    float4 x0, x1;
    float y, w;
    bool ok;
};

template <bool TRAIN>
__device__ inline RowIn fetch_row(const MlpArgs& a, int64_t rr, int kg)
{
    RowIn d;
    d.ok = rr < a.R;
    const int64_t row = mlp_row(a, d.ok ? rr : a.R - 1);
    const float4* x = reinterpret_cast<const float4*>(a.X + row * kF + 8 * kg);
    d.x0 = x[0];
    d.x1 = x[1];
    d.y = TRAIN ? a.y[row] : 0.f;
    d.w = TRAIN ? a.w[row] : 0.f;
    return d;
}

// (x - mean) / std of features 8kg .. 8kg + 7 as bf16 pairs
__device__ inline void normalise(const RowIn& in, const float* pb, int kg, uint32_t xp[4])
{
    const float xf[8] = {in.x0.x, in.x0.y, in.x0.z, in.x0.w, in.x1.x, in.x1.y, in.x1.z, in.x1.w};
    const float4 m0 = *reinterpret_cast<const float4*>(pb + pMean + 8 * kg);
    const float4 m1 = *reinterpret_cast<const float4*>(pb + pMean + 8 * kg + 4);
    const float4 s0 = *reinterpret_cast<const float4*>(pb + pInv + 8 * kg);
    const float4 s1 = *reinterpret_cast<const float4*>(pb + pInv + 8 * kg + 4);
    const float mf[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
    const float sf[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
        xp[j] = pack_bf16((xf[2 * j] - mf[2 * j]) * sf[2 * j], (xf[2 * j + 1] - mf[2 * j + 1]) * sf[2 * j + 1]);
}

// Layer 1, units 16t + 4kg + v of the lane's row: h1 (bf16 pairs) and, for
// training, gelu'(z1).
template <bool GP>
__device__ inline void layer1_tile(const bf16_t* w1t, const float* pb, bf16x8 xb, int t, int i16, int kg,
                                   uint32_t hp[2], float gp[4])
{
    const f32x4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_bf16x8(sw32(w1t, 16 * t + i16, 8 * kg)), xb,
                                                           f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    const float4 b = *reinterpret_cast<const float4*>(pb + pB1 + 16 * t + 4 * kg);
    const float bias[4] = {b.x, b.y, b.z, b.w};
    float h[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) gelu_terms<GP>(z[v] + bias[v], h[v], gp[v]);
    hp[0] = pack_bf16(h[0], h[1]);
    hp[1] = pack_bf16(h[2], h[3]);
}

// sum over K of W[16n + i16][K] x act[K] for the lane's row: W in LDS
// (swizzled, fragment order), act = the previous product's bf16 pairs by tile
__device__ inline f32x4 hidden_product(const bf16_t* w, const uint32_t (*ap)[2], int n, int i16, int kg)
{
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint4 bq = make_uint4(ap[2 * c][0], ap[2 * c][1], ap[2 * c + 1][0], ap[2 * c + 1][1]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_bf16x8(sw128(w, 16 * n + i16, 32 * c + 8 * kg)),
                                                      __builtin_bit_cast(bf16x8, bq), acc, 0, 0, 0);
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Forward only: one 128-row tile per workgroup.
struct FwdLds {
    bf16_t w1t[kH * kF];
    bf16_t w2p[kH * kH];
    float pb[kPb];
};

__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_forward(const MlpArgs a)
{
    __shared__ __align__(16) FwdLds L;
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, kg = lane >> 4;
    const int64_t rr = (int64_t)blockIdx.x * kMlpRows + 16 * wid + i16;
    const RowIn in = fetch_row<false>(a, rr, kg);
    stage_weights<false>(a, L.w1t, L.w2p, nullptr, L.pb);
    __syncthreads();

    uint32_t xp[4];
    normalise(in, L.pb, kg, xp);
    const bf16x8 xb = __builtin_bit_cast(bf16x8, make_uint4(xp[0], xp[1], xp[2], xp[3]));
    uint32_t h1p[8][2];
    float unused[4];
#pragma unroll
    for (int t = 0; t < 8; ++t) layer1_tile<false>(L.w1t, L.pb, xb, t, i16, kg, h1p[t], unused);
    float outp = 0.f;
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const f32x4 acc = hidden_product(L.w2p, h1p, n, i16, kg);
        const float4 b2 = *reinterpret_cast<const float4*>(L.pb + pB2 + 16 * n + 4 * kg);
        const float4 w3 = *reinterpret_cast<const float4*>(L.pb + pW3 + 16 * n + 4 * kg);
        const float bias[4] = {b2.x, b2.y, b2.z, b2.w}, w3v[4] = {w3.x, w3.y, w3.z, w3.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float h, g;
            gelu_terms<false>(acc[v] + bias[v], h, g);
            outp += h * w3v[v];
        }
    }
    outp += __shfl_xor(outp, 16);
    outp += __shfl_xor(outp, 32);
    if (kg == 0 && rr < a.R) a.out[rr] = outp + L.pb[pB3];
}

// ---------------------------------------------------------------------------
// One training step's gradient: forward, backward and weight gradients fused.
//
// One workgroup per compute unit loops over the step's 128-row tiles (wave w:
// rows 16w .. 16w + 15).  Per tile: the forward layers, the loss gradient,
// layer 3 backward and the layer-2 dgrad in registers (as in the forward
// kernel); the tile's Xn, h1, dz2 and then dz1 go to LDS transposed ([unit]
// [row], bf16), where the weight-gradient products take them with the rows
// as K: wave w adds dW2[:, 16w .. 16w + 15] = h1^T dz2 and
// dW1[:, 16w .. 16w + 15] = Xn^T dz1 to accumulators that stay in registers
// over all its tiles.  Bias, w3, b3 and loss sums: per wave in LDS (fp32, 16
// rows at a time).  The next tile's rows are requested while the current one
// is computed.  At the end the workgroup writes one partial row (dW1 | dW2 |
// sums) for the update kernel.
struct TrainLds {
    bf16_t w1t[kH * kF];
    bf16_t w2p[kH * kH];
    bf16_t w2q[kH * kH];
    bf16_t hT[kH * kMlpRows];   // h1^T of the tile, then dz1^T
    bf16_t dT[kH * kMlpRows];   // dz2^T
    bf16_t xT[kF * kMlpRows];   // Xn^T
    float pb[kPb];
    float part[kMlpWaves][kPartLd];
};

__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_train(const MlpArgs a)
{
    __shared__ __align__(16) TrainLds L;
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, kg = lane >> 4, qa = i16 >> 2, qb = i16 & 3;
    const int r0 = 16 * wid;   // the wave's first row in a tile
    const int ntiles = (a.R + kMlpRows - 1) / kMlpRows;
    RowIn cur = fetch_row<true>(a, (int64_t)blockIdx.x * kMlpRows + r0 + i16, kg);
    for (int k = lane; k < kPartLd; k += 64) L.part[wid][k] = 0.f;
    stage_weights<true>(a, L.w1t, L.w2p, L.w2q, L.pb);
    __syncthreads();
    float* part = L.part[wid];

    f32x4 acc2[8], acc1[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    acc1[0] = acc1[1] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // ---- normalised features (layer 1's B operand; Xn^T to LDS)
        uint32_t xp[4];
        normalise(cur, L.pb, kg, xp);
        put_transposed(L.xT, 8 * kg + qb, r0 + 4 * qa, xp[0], xp[1], qb);
        put_transposed(L.xT, 8 * kg + 4 + qb, r0 + 4 * qa, xp[2], xp[3], qb);
        // a row past the end has weight 0: no loss and no gradient
        const float yv = cur.y, wv = cur.ok ? cur.w : 0.f;
        if (tile + (int)gridDim.x < ntiles)
            cur = fetch_row<true>(a, (int64_t)(tile + gridDim.x) * kMlpRows + r0 + i16, kg);
        const bf16x8 xb = __builtin_bit_cast(bf16x8, make_uint4(xp[0], xp[1], xp[2], xp[3]));

        // ---- layer 1 (h1^T to LDS)
        uint32_t h1p[8][2];
        float gp1[8][4];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            layer1_tile<true>(L.w1t, L.pb, xb, t, i16, kg, h1p[t], gp1[t]);
            put_transposed(L.hT, 16 * t + 4 * kg + qb, r0 + 4 * qa, h1p[t][0], h1p[t][1], qb);
        }

        // ---- layer 2 and the output (fp32)
        float h2[8][4], gp2[8][4];
        float outp = 0.f;
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            const f32x4 acc = hidden_product(L.w2p, h1p, n, i16, kg);
            const float4 b2 = *reinterpret_cast<const float4*>(L.pb + pB2 + 16 * n + 4 * kg);
            const float4 w3 = *reinterpret_cast<const float4*>(L.pb + pW3 + 16 * n + 4 * kg);
            const float bias[4] = {b2.x, b2.y, b2.z, b2.w}, w3v[4] = {w3.x, w3.y, w3.z, w3.w};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                gelu_terms<true>(acc[v] + bias[v], h2[n][v], gp2[n][v]);
                outp += h2[n][v] * w3v[v];
            }
        }
        outp += __shfl_xor(outp, 16);
        outp += __shfl_xor(outp, 32);
        const float diff = outp + L.pb[pB3] - yv;
        const float dout = 2.0f * wv * diff * a.inv_denom;
        const float lossp = wv * diff * diff * a.inv_denom;

        // ---- layer 3 backward, layer 2 deltas (dz2^T to LDS), b2 and w3 sums
        uint32_t dz2p[8][2];
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            const float4 w3 = *reinterpret_cast<const float4*>(L.pb + pW3 + 16 * n + 4 * kg);
            const float w3v[4] = {w3.x, w3.y, w3.z, w3.w};
            float d[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) d[v] = dout * w3v[v] * gp2[n][v];
            dz2p[n][0] = pack_bf16(d[0], d[1]);
            dz2p[n][1] = pack_bf16(d[2], d[3]);
            put_transposed(L.dT, 16 * n + 4 * kg + qb, r0 + 4 * qa, dz2p[n][0], dz2p[n][1], qb);
            // unit 16n + 4kg + qb's sums (the row's four quads write the same value)
            part[kH + 16 * n + 4 * kg + qb] += row16_sum4(d[0], d[1], d[2], d[3], qb);
            part[2 * kH + 16 * n + 4 * kg + qb] +=
                row16_sum4(h2[n][0] * dout, h2[n][1] * dout, h2[n][2] * dout, h2[n][3] * dout, qb);
        }

        // ---- dgrad of layer 2 (dh1^T = W2 dz2^T) through GELU; b1 sums
        uint32_t dz1p[8][2];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const f32x4 acc = hidden_product(L.w2q, dz2p, t, i16, kg);
            float d[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) d[v] = acc[v] * gp1[t][v];
            dz1p[t][0] = pack_bf16(d[0], d[1]);
            dz1p[t][1] = pack_bf16(d[2], d[3]);
            part[16 * t + 4 * kg + qb] += row16_sum4(d[0], d[1], d[2], d[3], qb);
        }
        // b3 and the loss (quad lanes 0 and 1; lanes 2 and 3 add zeros to the
        // padding after them)
        part[3 * kH + qb] += row16_sum4(dout, lossp, 0.f, 0.f, qb);
        __syncthreads();

        // ---- dW2[:, 16w ..] += h1^T dz2 over the tile's 128 rows
        {
            bf16x8 bq[4];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) bq[ks] = lds_bf16x8(sw128(L.dT, r0 + i16, 32 * ks + 8 * kg));
#pragma unroll
            for (int it = 0; it < 8; ++it)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    acc2[it] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        lds_bf16x8(sw128(L.hT, 16 * it + i16, 32 * ks + 8 * kg)), bq[ks], acc2[it], 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8; ++t) put_transposed(L.hT, 16 * t + 4 * kg + qb, r0 + 4 * qa, dz1p[t][0], dz1p[t][1], qb);
        __syncthreads();

        // ---- dW1[:, 16w ..] += Xn^T dz1
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8 bq = lds_bf16x8(sw128(L.hT, r0 + i16, 32 * ks + 8 * kg));
#pragma unroll
            for (int ft = 0; ft < 2; ++ft)
                acc1[ft] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    lds_bf16x8(sw128(L.xT, 16 * ft + i16, 32 * ks + 8 * kg)), bq, acc1[ft], 0, 0, 0);
        }
        __syncthreads();
    }

    // ---- the workgroup's partial row: lane (o = 16w + i16, kg) holds rows
    // 16it + 4kg + v of dW2 and 16ft + 4kg + v of dW1
    float* dst = a.wpart + (int64_t)blockIdx.x * kWRow;
#pragma unroll
    for (int it = 0; it < 8; ++it)
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[oW2 + (16 * it + 4 * kg + v) * kH + r0 + i16] = acc2[it][v];
#pragma unroll
    for (int ft = 0; ft < 2; ++ft)
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[oW1 + (16 * ft + 4 * kg + v) * kH + r0 + i16] = acc1[ft][v];
    for (int k = threadIdx.x; k < kPart; k += blockDim.x) {
        float t = L.part[0][k];
#pragma unroll
        for (int w = 1; w < kMlpWaves; ++w) t += L.part[w][k];
        dst[ob2 + k] = t;
    }
}

struct UpdateArgs {
    float* P;                // master parameters
    float* m;                // Adam first moments
    float* v;                // Adam second moments
    float* grads;            // the assembled gradient [kParams]
    const float* wpart;      // partial rows [nks][kWRow]
    int32_t nks;
    int32_t apply;           // 0: only assemble the gradient
    float lr, beta1, beta2, eps;
    float bc1, bc2;          // 1 - beta^t
    bf16_t* W1T;
    bf16_t* W2T;
    bf16_t* W2;
    float* loss_out;         // loss of this step, or null
};

// Gradient assembly and Adam: 128 parameters per workgroup (one round of
// workgroups over the device), eight threads per parameter, thread q summing
// the partial rows q, q + 8, ... in 32 interleaved running sums (all its
// loads in flight at once for up to 256 partial rows) joined pairwise in a
// fixed order, the eight threads' sums then added in a fixed order.  Index
// kParams is the loss.
constexpr int kUpdParams = 128, kUpdSlices = 8, kUpdAcc = 32;

__device__ inline float strided_sum(const float* base, int64_t stride, int count, int q)
{
    float acc[kUpdAcc];
#pragma unroll
    for (int j = 0; j < kUpdAcc; ++j) acc[j] = 0.f;
    int k = q;
    for (; k + (kUpdAcc - 1) * kUpdSlices < count; k += kUpdAcc * kUpdSlices)
#pragma unroll
        for (int j = 0; j < kUpdAcc; ++j) acc[j] += base[(int64_t)(k + j * kUpdSlices) * stride];
    for (int j = 0; k < count; k += kUpdSlices, ++j) acc[j] += base[(int64_t)k * stride];
#pragma unroll
    for (int h = kUpdAcc / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int j = 0; j < h; ++j) acc[j] += acc[j + h];
    return acc[0];
}

__global__ __launch_bounds__(1024) void k_mlp_update(const UpdateArgs u)
{
    __shared__ float red[kUpdSlices][kUpdParams];
    const int c = threadIdx.x % kUpdParams, q = threadIdx.x / kUpdParams;
    const int p = blockIdx.x * kUpdParams + c;
    float s = 0.f;
    if (p <= kParams) {
        int col;
        if ((p >= oW1 && p < ob1) || (p >= oW2 && p < ob2))
            col = p;
        else if (p == kParams)
            col = ob2 + 3 * kH + 1;        // loss
        else if (p < oW2)
            col = ob2 + (p - ob1);         // db1
        else if (p < ow3)
            col = ob2 + kH + (p - ob2);    // db2
        else if (p < ob3)
            col = ob2 + 2 * kH + (p - ow3); // dw3
        else
            col = ob2 + 3 * kH;            // db3
        s = strided_sum(u.wpart + col, kWRow, u.nks, q);
    }
    red[q][c] = s;
    __syncthreads();
    if (q != 0 || p > kParams) return;
    float g = 0.f;
#pragma unroll
    for (int t = 0; t < kUpdSlices; ++t) g += red[t][c];
    if (p == kParams) {
        if (u.loss_out) *u.loss_out = g;
        return;
    }
    u.grads[p] = g;
    if (!u.apply) return;
    const float m = u.beta1 * u.m[p] + (1.0f - u.beta1) * g;
    const float v = u.beta2 * u.v[p] + (1.0f - u.beta2) * g * g;
    u.m[p] = m;
    u.v[p] = v;
    const float mh = m / u.bc1, vh = v / u.bc2;
    const float np = u.P[p] - u.lr * mh / (sqrtf(vh) + u.eps);
    u.P[p] = np;
    if (p < ob1) {
        const int f = p / kH, o = p % kH;
        u.W1T[o * kF + f] = to_bf16(np);
    } else if (p >= oW2 && p < ob2) {
        const int i = (p - oW2) / kH, o = (p - oW2) % kH;
        u.W2[i * kH + o] = to_bf16(np);
        u.W2T[o * kH + i] = to_bf16(np);
    }
}

__global__ __launch_bounds__(256) void k_mlp_bf16_copies(const float* P, bf16_t* W1T, bf16_t* W2T, bf16_t* W2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < ob1) {
        const int f = p / kH, o = p % kH;
        W1T[o * kF + f] = to_bf16(P[p]);
    } else if (p >= oW2 && p < ob2) {
        const int i = (p - oW2) / kH, o = (p - oW2) % kH;
        W2[i * kH + o] = to_bf16(P[p]);
        W2T[o * kH + i] = to_bf16(P[p]);
    }
}

}  // namespace mcinv

using namespace mcinv;

struct mcinv_mlp {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    float* P = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* grads = nullptr;
    bf16_t* W1T = nullptr;
    bf16_t* W2T = nullptr;
    bf16_t* W2 = nullptr;
    float* mean = nullptr;
    float* inv_std = nullptr;
    int64_t t = 0;           // Adam steps taken
    // training data
    float* X = nullptr;
    float* y = nullptr;
    float* w = nullptr;
    int64_t N = 0;
    // step buffers
    int32_t Rcap = 0;
    int32_t cus = 0;         // compute units: training workgroups per step (at most)
    float* wpart = nullptr;  // [cus][kWRow]
    int64_t* idx = nullptr;
    float* loss = nullptr;
    std::string err;
};

namespace {

thread_local std::string g_merr;

template <typename T>
void mfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

mcinv_status merr(mcinv_mlp* m, mcinv_status code, const std::string& msg)
{
    if (m)
        m->err = msg;
    else
        g_merr = msg;
    return code;
}

#define MHIP(m, expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return merr((m), e_ == hipErrorOutOfMemory ? MCINV_ENOMEM : MCINV_EDEVICE,          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                     \
    } while (0)

mcinv_status ensure_step(mcinv_mlp* m, int32_t R)
{
    if (R <= m->Rcap) return MCINV_OK;
    m->Rcap = 0;   // until the row list is allocated again
    mfree(m->idx);
    MHIP(m, hipMalloc((void**)&m->idx, sizeof(int64_t) * R));
    m->Rcap = R;
    return MCINV_OK;
}

MlpArgs base_args(mcinv_mlp* m)
{
    MlpArgs a{};
    a.mean = m->mean;
    a.inv_std = m->inv_std;
    a.W1T = m->W1T;
    a.W2T = m->W2T;
    a.W2 = m->W2;
    a.P = m->P;
    return a;
}

// One training step over R rows: the fused kernel (one partial row per
// workgroup, at most one workgroup per compute unit), then the gradient
// assembly and, with `apply`, the Adam step.  The rows: drawn from Philox
// (key = seed, counter word 1 = the step about to be taken) with `draw`,
// else the list in m->idx.
mcinv_status run_step(mcinv_mlp* m, int32_t R, bool apply, float lr, float* loss_dev, bool draw = false,
                      uint64_t seed = 0)
{
    MlpArgs a = base_args(m);
    a.X = m->X;
    a.y = m->y;
    a.w = m->w;
    a.idx = m->idx;
    a.draw = draw ? 1 : 0;
    a.key0 = (uint32_t)(seed & 0xffffffffu);
    a.key1 = (uint32_t)(seed >> 32);
    a.step = (uint32_t)(m->t + 1);
    a.N = m->N;
    a.R = R;
    a.wpart = m->wpart;
    a.inv_denom = 1.0f / (float)R;
    const int32_t nks = std::min((R + kMlpRows - 1) / kMlpRows, m->cus);
    k_mlp_train<<<dim3(nks), dim3(64 * kMlpWaves), 0, m->stream>>>(a);
    MHIP(m, hipGetLastError());
    UpdateArgs u{};
    u.P = m->P;
    u.m = m->m;
    u.v = m->v;
    u.grads = m->grads;
    u.wpart = m->wpart;
    u.nks = nks;
    u.apply = apply ? 1 : 0;
    u.lr = lr;
    u.beta1 = 0.9f;
    u.beta2 = 0.999f;
    u.eps = 1e-8f;
    if (apply) {
        m->t += 1;
        u.bc1 = 1.0f - powf(0.9f, (float)m->t);
        u.bc2 = 1.0f - powf(0.999f, (float)m->t);
    } else {
        u.bc1 = u.bc2 = 1.0f;
    }
    u.W1T = m->W1T;
    u.W2T = m->W2T;
    u.W2 = m->W2;
    u.loss_out = loss_dev;
    k_mlp_update<<<dim3((kParams + kUpdParams) / kUpdParams), dim3(kUpdParams * kUpdSlices), 0, m->stream>>>(u);
    MHIP(m, hipGetLastError());
    return MCINV_OK;
}

}  // namespace

namespace mcinv {

mcinv_status mlp_predict_device(mcinv_mlp* m, const float* dX, int64_t N, float* dout, std::string* err)
{
    hipError_t e = hipSuccess;
    const int64_t chunk = (int64_t)64 * 65535;
    for (int64_t r0 = 0; r0 < N && e == hipSuccess; r0 += chunk) {
        MlpArgs a = base_args(m);
        a.X = dX;
        a.idx = nullptr;
        a.row0 = r0;
        a.R = (int32_t)std::min<int64_t>(chunk, N - r0);
        a.out = dout + r0;
        k_mlp_forward<<<dim3((unsigned)((a.R + kMlpRows - 1) / kMlpRows)), dim3(64 * kMlpWaves), 0, m->stream>>>(a);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return MCINV_EDEVICE;
    }
    return MCINV_OK;
}

}  // namespace mcinv

extern "C" {

mcinv_status mcinv_mlp_create(int32_t device, mcinv_mlp** out)
try {
    if (!out) return merr(nullptr, MCINV_EINVAL, "null argument");
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return merr(nullptr, MCINV_EDEVICE, "no such device");
    // the owner destroys a partly built network on every early return or exception
    std::unique_ptr<mcinv_mlp, void (*)(mcinv_mlp*)> owner(new mcinv_mlp(), mcinv_mlp_destroy);
    mcinv_mlp* m = owner.get();
    m->device = device;
    auto fail_alloc = [&]() {
        return merr(nullptr, MCINV_ENOMEM, "device allocation failed");
    };
    if (hipStreamCreate(&m->stream) != hipSuccess) return fail_alloc();
    if (hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || m->cus < 1)
        return merr(nullptr, MCINV_EDEVICE, "cannot read the device's compute unit count");
    if (hipMalloc((void**)&m->wpart, sizeof(float) * kWRow * (size_t)m->cus) != hipSuccess ||
        hipMalloc((void**)&m->P, sizeof(float) * kParams) != hipSuccess ||
        hipMalloc((void**)&m->m, sizeof(float) * kParams) != hipSuccess ||
        hipMalloc((void**)&m->v, sizeof(float) * kParams) != hipSuccess ||
        hipMalloc((void**)&m->grads, sizeof(float) * kParams) != hipSuccess ||
        hipMalloc((void**)&m->W1T, sizeof(bf16_t) * kF * kH) != hipSuccess ||
        hipMalloc((void**)&m->W2T, sizeof(bf16_t) * kH * kH) != hipSuccess ||
        hipMalloc((void**)&m->W2, sizeof(bf16_t) * kH * kH) != hipSuccess ||
        hipMalloc((void**)&m->mean, sizeof(float) * kF) != hipSuccess ||
        hipMalloc((void**)&m->inv_std, sizeof(float) * kF) != hipSuccess ||
        hipMalloc((void**)&m->loss, sizeof(float) * 1) != hipSuccess)
        return fail_alloc();
    std::vector<float> zero(kParams, 0.0f), one(kF, 1.0f);
    if (hipMemcpy(m->P, zero.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->m, zero.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->v, zero.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->mean, zero.data(), sizeof(float) * kF, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->inv_std, one.data(), sizeof(float) * kF, hipMemcpyHostToDevice) != hipSuccess)
        return fail_alloc();
    *out = owner.release();
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(nullptr, s_, m_); });
}

void mcinv_mlp_destroy(mcinv_mlp* m)
{
    if (!m) return;
    (void)hipSetDevice(m->device);
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    mfree(m->P);
    mfree(m->m);
    mfree(m->v);
    mfree(m->grads);
    mfree(m->W1T);
    mfree(m->W2T);
    mfree(m->W2);
    mfree(m->mean);
    mfree(m->inv_std);
    mfree(m->loss);
    mfree(m->X);
    mfree(m->y);
    mfree(m->w);
    mfree(m->idx);
    mfree(m->wpart);
    if (m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
}

mcinv_status mcinv_mlp_set_params(mcinv_mlp* m, const float* params)
try {
    if (!m || !params) return merr(m, MCINV_EINVAL, "null argument");
    MHIP(m, hipSetDevice(m->device));
    MHIP(m, hipMemcpyAsync(m->P, params, sizeof(float) * kParams, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemsetAsync(m->m, 0, sizeof(float) * kParams, m->stream));
    MHIP(m, hipMemsetAsync(m->v, 0, sizeof(float) * kParams, m->stream));
    k_mlp_bf16_copies<<<dim3((kParams + 255) / 256), dim3(256), 0, m->stream>>>(m->P, m->W1T, m->W2T, m->W2);
    MHIP(m, hipGetLastError());
    MHIP(m, hipStreamSynchronize(m->stream));
    m->t = 0;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

mcinv_status mcinv_mlp_get_params(mcinv_mlp* m, float* params)
try {
    if (!m || !params) return merr(m, MCINV_EINVAL, "null argument");
    MHIP(m, hipSetDevice(m->device));
    MHIP(m, hipMemcpyAsync(params, m->P, sizeof(float) * kParams, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

mcinv_status mcinv_mlp_set_normalization(mcinv_mlp* m, const float* mean, const float* inv_std)
try {
    if (!m || !mean || !inv_std) return merr(m, MCINV_EINVAL, "null argument");
    MHIP(m, hipSetDevice(m->device));
    MHIP(m, hipMemcpyAsync(m->mean, mean, sizeof(float) * kF, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemcpyAsync(m->inv_std, inv_std, sizeof(float) * kF, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

mcinv_status mcinv_mlp_set_data(mcinv_mlp* m, const float* X, const float* y, const float* w, int64_t N)
try {
    if (!m || !X || !y || !w || N < 1) return merr(m, MCINV_EINVAL, "bad arguments");
    MHIP(m, hipSetDevice(m->device));
    mfree(m->X);
    mfree(m->y);
    mfree(m->w);
    MHIP(m, hipMalloc((void**)&m->X, sizeof(float) * kF * N));
    MHIP(m, hipMalloc((void**)&m->y, sizeof(float) * N));
    MHIP(m, hipMalloc((void**)&m->w, sizeof(float) * N));
    MHIP(m, hipMemcpyAsync(m->X, X, sizeof(float) * kF * N, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemcpyAsync(m->y, y, sizeof(float) * N, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemcpyAsync(m->w, w, sizeof(float) * N, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    m->N = N;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

mcinv_status mcinv_mlp_fit_normalization(mcinv_mlp* m, float* mean_out, float* inv_std_out)
try {
    if (!m) return merr(m, MCINV_EINVAL, "null argument");
    if (m->N < 1) return merr(m, MCINV_ESTATE, "no training data");
    MHIP(m, hipSetDevice(m->device));
    std::vector<float> X((size_t)m->N * kF);
    MHIP(m, hipMemcpyAsync(X.data(), m->X, sizeof(float) * X.size(), hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    float mean[kF], inv[kF];
    for (int k = 0; k < kF; ++k) {
        double s = 0.0;
        for (int64_t i = 0; i < m->N; ++i) s += (double)X[(size_t)i * kF + k];
        const double mu = s / (double)m->N;
        double v = 0.0;
        for (int64_t i = 0; i < m->N; ++i) {
            const double d = (double)X[(size_t)i * kF + k] - mu;
            v += d * d;
        }
        v /= (double)m->N;
        mean[k] = (float)mu;
        inv[k] = v > 1e-12 ? (float)(1.0 / std::sqrt(v)) : 1.0f;
    }
    if (mean_out) std::memcpy(mean_out, mean, sizeof(mean));
    if (inv_std_out) std::memcpy(inv_std_out, inv, sizeof(inv));
    return mcinv_mlp_set_normalization(m, mean, inv);
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

mcinv_status mcinv_mlp_label_weights(int64_t N, const double* y_se, double eps, float* w)
try {
    if (N < 1 || !y_se || !w || !(eps > 0.0)) return merr(nullptr, MCINV_EINVAL, "bad arguments");
    std::vector<double> raw(N);
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        if (!(y_se[i] >= 0.0) || !std::isfinite(y_se[i]))
            return merr(nullptr, MCINV_EINVAL, "label standard error must be finite and >= 0");
        raw[i] = 1.0 / (y_se[i] * y_se[i] + eps);
        s += raw[i];
    }
    const double scale = (double)N / s;
    for (int64_t i = 0; i < N; ++i) w[i] = (float)(raw[i] * scale);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(nullptr, s_, m_); });
}

mcinv_status mcinv_mlp_gradients(mcinv_mlp* m, const int64_t* rows, int32_t nrows, float* grads, float* loss)
try {
    if (!m || !rows || !grads) return merr(m, MCINV_EINVAL, "null argument");
    if (nrows < 64 || nrows % 64 != 0) return merr(m, MCINV_EINVAL, "nrows must be a positive multiple of 64");
    if (m->N < 1) return merr(m, MCINV_ESTATE, "no training data");
    for (int32_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= m->N) return merr(m, MCINV_EINVAL, "row index out of range");
    MHIP(m, hipSetDevice(m->device));
    {
        const mcinv_status st = ensure_step(m, nrows);
        if (st != MCINV_OK) return st;
    }
    MHIP(m, hipMemcpyAsync(m->idx, rows, sizeof(int64_t) * nrows, hipMemcpyHostToDevice, m->stream));
    mcinv_status s = run_step(m, nrows, false, 0.0f, m->loss);
    if (s != MCINV_OK) return s;
    MHIP(m, hipMemcpyAsync(grads, m->grads, sizeof(float) * kParams, hipMemcpyDeviceToHost, m->stream));
    float l = 0.f;
    MHIP(m, hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    if (loss) *loss = l;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

mcinv_status mcinv_mlp_train(mcinv_mlp* m, int64_t steps, int32_t batch_rows, float lr, uint64_t seed,
                             float* loss_history)
try {
    if (!m || steps < 0) return merr(m, MCINV_EINVAL, "bad arguments");
    if (batch_rows < 64 || batch_rows % 64 != 0 || batch_rows > (1 << 20))
        return merr(m, MCINV_EINVAL, "batch_rows must be a multiple of 64 in [64, 2^20]");
    if (m->N < 1) return merr(m, MCINV_ESTATE, "no training data");
    MHIP(m, hipSetDevice(m->device));
    {
        const mcinv_status st = ensure_step(m, batch_rows);
        if (st != MCINV_OK) return st;
    }
    struct LossBuf {  // freed on every return path (hipFree waits for the device)
        float* p = nullptr;
        ~LossBuf() { mfree(p); }
    } dloss;
    if (loss_history && steps > 0) MHIP(m, hipMalloc((void**)&dloss.p, sizeof(float) * steps));
    for (int64_t s = 0; s < steps; ++s) {
        const mcinv_status st = run_step(m, batch_rows, true, lr, dloss.p ? dloss.p + s : nullptr, true, seed);
        if (st != MCINV_OK) return st;
    }
    if (dloss.p)
        MHIP(m, hipMemcpyAsync(loss_history, dloss.p, sizeof(float) * steps, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

mcinv_status mcinv_mlp_predict(mcinv_mlp* m, const float* X, int64_t N, float* out)
try {
    if (!m || !X || !out || N < 0) return merr(m, MCINV_EINVAL, "bad arguments");
    if (N == 0) return MCINV_OK;
    MHIP(m, hipSetDevice(m->device));
    float *dX = nullptr, *dout = nullptr;
    MHIP(m, hipMalloc((void**)&dX, sizeof(float) * kF * N));
    if (hipMalloc((void**)&dout, sizeof(float) * N) != hipSuccess) {
        mfree(dX);
        return merr(m, MCINV_ENOMEM, "device allocation failed");
    }
    std::string why;
    mcinv_status st = MCINV_OK;
    hipError_t e = hipMemcpyAsync(dX, X, sizeof(float) * kF * N, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) st = mcinv::mlp_predict_device(m, dX, N, dout, &why);
    if (e == hipSuccess && st == MCINV_OK)
        e = hipMemcpyAsync(out, dout, sizeof(float) * N, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess && st == MCINV_OK) e = hipStreamSynchronize(m->stream);
    mfree(dX);
    mfree(dout);
    if (st != MCINV_OK) return merr(m, st, "predict: " + why);
    if (e != hipSuccess) return merr(m, MCINV_EDEVICE, std::string("predict: ") + hipGetErrorString(e));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

mcinv_status mcinv_mlp_estimate_matrix(mcinv_mlp* m, const mcinv_gate* g, int64_t n, int64_t nnz,
                                       const int64_t* row_ptr, const int32_t* col_idx, const double* values,
                                       double* est, uint8_t* fallback)
try {
    if (!m || !g || !est || !fallback) return merr(m, MCINV_EINVAL, "estimate_matrix: null argument");
    std::string why;
    float* dF = nullptr;
    float* dout = nullptr;
    struct Release {   // the two device buffers, on every exit
        float** a;
        float** b;
        ~Release()
        {
            if (*a) (void)hipFree(*a);
            if (*b) (void)hipFree(*b);
        }
    } release{&dF, &dout};
    std::vector<double> diag;
    mcinv_status st = mcinv::features_on_device(m->device, n, nnz, row_ptr, col_idx, values, &dF, &why, &diag);
    if (st != MCINV_OK) return merr(m, st, "estimate_matrix: features: " + why);
    std::vector<float> pred((size_t)n);
    std::vector<float> two;
    if (hipMalloc((void**)&dout, sizeof(float) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) {
        dout = nullptr;
        st = MCINV_ENOMEM;
        why = "device allocation failed";
    }
    if (st == MCINV_OK) st = mcinv::mlp_predict_device(m, dF, n, dout, &why);
    if (st == MCINV_OK && hipMemcpy(pred.data(), dout, sizeof(float) * n, hipMemcpyDeviceToHost) != hipSuccess) {
        st = MCINV_EDEVICE;
        why = "copying the predictions failed";
    }
    if (st == MCINV_OK) {
        two.resize((size_t)n * 2);
        st = mcinv::features_pick_two(dF, n, mcinv::gate_feature_a(g), mcinv::gate_feature_b(g), two.data(), &why);
    }
    if (st != MCINV_OK) return merr(m, st, "estimate_matrix: " + why);
    mcinv::gate_fallback_rows(g, n, two.data(), 2, 0, 1, fallback);
    for (int64_t i = 0; i < n; ++i) {
        est[i] = (double)pred[i] / diag[i];   // the network predicts c_ii (C^-1)_ii
        if (!std::isfinite(pred[i])) fallback[i] = 1;
    }
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { merr(m, s_, m_); });
}

const char* mcinv_mlp_last_error(const mcinv_mlp* m)
{
    return m ? m->err.c_str() : g_merr.c_str();
}

}  // extern "C"
