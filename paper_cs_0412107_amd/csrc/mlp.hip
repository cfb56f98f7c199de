// The learned surrogate's network: MLP 32 -> 128 -> 128 -> 1 with GELU
// (erf form), bf16 operands on the matrix cores with fp32 accumulation, fp32
// master weights and Adam (Kingma & Ba, 2015).  It predicts y_i = c_ii
// (C^-1)_ii from the 32 local features of row i.
//
// Kernels
//   k_mlp_fwd_bwd : one wave = 16 rows.  Layer 1 and 2 products on
//                   v_mfma_f32_16x16x32_bf16 (A = activations, B = weights
//                   from global), GELU in fp32, output layer in fp32.  The
//                   training instance (BWD): the weighted-MSE gradient flows back through
//                   layer 3 (fp32), layer 2 (dgrad on MFMA) and both GELUs;
//                   activations and deltas go out transposed as bf16 for the
//                   weight gradients, bias / w3 partial sums per workgroup.
//   k_mlp_wgrad   : dW1 = X^T dz1, dW2 = h1^T dz2 over the step's rows
//                   (the whole 128 x 128 or 32 x 128 output per workgroup,
//                   one sub-tile per wave, the rows split over workgroups).
//   k_mlp_update  : gradient assembly (every partial summed in a fixed
//                   order), Adam step, bf16 copies of the weights.
// Training draws each step's rows from Philox inside k_mlp_fwd_bwd.
// Rounding points (what the oracle reproduces): the normalised features,
// W1, W2, h1 and dz2 enter MFMA products as bf16 (nearest even); h2, w3, the
// biases and every elementwise step stay fp32.
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
constexpr int kActLd = kH + 8;       // LDS row pitch (bf16) of one wave's activations
constexpr int kWRow = ob2 + kPart;   // one weight-gradient partial row: W1 | b1 gap | W2 | block sums

typedef unsigned short bf16_t;

// round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ inline bf16_t to_bf16(float x) { return __builtin_bit_cast(bf16_t, (__bf16)x); }

__device__ inline bf16x8 load_bf16x8(const bf16_t* p)
{
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(bf16x8, u);
}

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
    bf16_t* XT;              // [32][R]
    bf16_t* h1T;             // [128][R]
    bf16_t* dz2T;            // [128][R]
    bf16_t* dz1T;            // [128][R]
    float* part;             // [blocks][kPart]
    float inv_denom;         // loss = sum_r w_r (out_r - y_r)^2 * inv_denom
};

// Write a wave's 16 rows x ncols block (bf16, row-major in LDS) to the
// transposed buffer dst[col][R] at rows r0w..r0w+15: lane l takes columns
// l, l + 64, ... and stores each column's 16 values as one 32-byte segment
// (r0w is a multiple of 16 and R a multiple of 64, so segments are aligned).
__device__ inline void store_transposed(const bf16_t (*src)[kActLd], int ncols, bf16_t* dst, int64_t R, int64_t r0w,
                                        int lane)
{
    for (int c = lane; c < ncols; c += 64) {
        u16x8 lo, hi;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            lo[r] = src[r][c];
            hi[r] = src[8 + r][c];
        }
        uint4* d = reinterpret_cast<uint4*>(dst + (int64_t)c * R + r0w);
        d[0] = __builtin_bit_cast(uint4, lo);
        d[1] = __builtin_bit_cast(uint4, hi);
    }
}

// GELU (erf form) and its derivative at z: h = z Phi(z) and gp = Phi(z) +
// z phi(z), with Phi(z) = (1 + erf(z / sqrt 2)) / 2 and phi(z) = exp(-z^2 / 2)
// / sqrt(2 pi).
template <bool GP>
__device__ inline void gelu_terms(float z, float& h, float& gp)
{
    constexpr float kRs2 = 0.70710678118654752f, kRs2pi = 0.39894228040143268f;
    const float e = erff(z * kRs2);
    h = 0.5f * z * (1.0f + e);
    gp = GP ? 0.5f * (1.0f + e) + z * expf(-0.5f * z * z) * kRs2pi : 0.0f;
}

// The four rows 4kg .. 4kg+3 of column c that a lane holds in an MFMA result
// (bf16) into the transposed buffer dst[c][R] at rows r0w + 4kg .. (8 bytes;
// r0w is a multiple of 16, so the store is aligned).
__device__ inline void store_col4(bf16_t* dst, int64_t R, int64_t r0w, int c, int kg, const bf16_t v[4])
{
    uint2 w;
    w.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
    w.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
    *reinterpret_cast<uint2*>(dst + (int64_t)c * R + r0w + 4 * kg) = w;
}

// Orders a wave's own LDS accesses (each wave works in its private slice of
// the workgroup's LDS, so no workgroup barrier is needed between its phases).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

#ifndef MCINV_MLP_MIN_BLOCKS
#define MCINV_MLP_MIN_BLOCKS 2   // workgroups per CU the register budget is sized for
#endif
template <bool BWD>
__global__ __launch_bounds__(256, MCINV_MLP_MIN_BLOCKS) void k_mlp_fwd_bwd(const MlpArgs a)
{
    // act (wave-private): the normalised features (written out transposed
    // for the weight gradients), then h1 (bf16) as layer 2's A operand, then
    // dz2 (bf16) as the dgrad A operand.  h1, dz2 and dz1 also go straight
    // from the MFMA result layout to their transposed buffers.  gelu'(z1)
    // and layer 2's GELU values stay in registers for the backward pass.
    __shared__ __align__(16) bf16_t act[4][16][kActLd];
    __shared__ float part[4][kPart];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int i16 = lane & 15, kg = lane >> 4;
    const int64_t r0w = (int64_t)blockIdx.x * 64 + wid * 16;
    const float* P = a.P;

    // ---- layer 1: A = normalised features (row i16, features 8kg..8kg+7)
    const int64_t ra = r0w + i16;
    const bool aok = ra < a.R;
    const int64_t rowa = aok ? mlp_row(a, ra) : 0;
    bf16x8 a1;
    {
        u16x8 u;
        const float* x = a.X + rowa * kF + 8 * kg;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float xn = aok ? (x[e] - a.mean[8 * kg + e]) * a.inv_std[8 * kg + e] : 0.0f;
            u[e] = to_bf16(xn);
            if (BWD) act[wid][i16][8 * kg + e] = u[e];
        }
        a1 = __builtin_bit_cast(bf16x8, u);
    }
    if (BWD) {   // backward launches cover whole 64-row blocks
        wave_lds_sync();
        store_transposed(act[wid], kF, a.XT, a.R, r0w, lane);
        wave_lds_sync();
    }
    // z1 -> h1 = GELU(z1) into LDS (bf16) and h1^T; gelu'(z1) kept in registers
    float gp1[8][4];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const bf16x8 b = load_bf16x8(a.W1T + (16 * n + i16) * kF + 8 * kg);
        const f32x4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        const float bias = P[ob1 + 16 * n + i16];
        bf16_t hb[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float hv, gv;
            gelu_terms<BWD>(z[v] + bias, hv, gv);
            hb[v] = to_bf16(hv);
            act[wid][4 * kg + v][16 * n + i16] = hb[v];
            gp1[n][v] = gv;
        }
        if (BWD) store_col4(a.h1T, a.R, r0w, 16 * n + i16, kg, hb);
        __builtin_amdgcn_sched_barrier(0);
    }
    wave_lds_sync();

    // ---- layer 2, and layer 3 (fp32) on the fly: out_v for rows r0w + 4kg + v
    float h2[8][4], gp2[8][4];
    float out[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&act[wid][i16][32 * s + 8 * kg]));
            const bf16x8 b = load_bf16x8(a.W2T + (16 * n + i16) * kH + 32 * s + 8 * kg);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, acc, 0, 0, 0);
        }
        const float bias = P[ob2 + 16 * n + i16];
        const float w3 = P[ow3 + 16 * n + i16];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            gelu_terms<BWD>(acc[v] + bias, h2[n][v], gp2[n][v]);
            out[v] += h2[n][v] * w3;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        for (int off = 1; off < 16; off <<= 1) out[v] += __shfl_xor(out[v], off);
        out[v] += P[ob3];
    }
    if (!BWD) {
        if (i16 == 0)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t rd = r0w + 4 * kg + v;
                if (rd < a.R) a.out[rd] = out[v];
            }
        return;
    }

    // ---- loss gradient (the rows 4kg + v of this lane's group: their data
    // rows come from the lanes i16 = 4kg + v that loaded them)
    float dout[4], lossp = 0.f, db3 = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t rd = r0w + 4 * kg + v;
        const int64_t row = __shfl(rowa, 4 * kg + v);
        float dv = 0.f;
        if (rd < a.R) {
            const float diff = out[v] - a.y[row];
            dv = 2.0f * a.w[row] * diff * a.inv_denom;
            lossp += a.w[row] * diff * diff * a.inv_denom;
        }
        dout[v] = dv;
        db3 += dv;
    }

    // ---- layer 3 backward and layer 2 deltas, written to LDS (bf16); every
    // lane has finished reading h1 (wave order)
    float dw3p[8], db2p[8];
    wave_lds_sync();
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const float w3 = P[ow3 + 16 * n + i16];
        float s3 = 0.f, s2 = 0.f;
        bf16_t db[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            s3 += h2[n][v] * dout[v];
            const float d = dout[v] * w3 * gp2[n][v];
            s2 += d;
            db[v] = to_bf16(d);
            act[wid][4 * kg + v][16 * n + i16] = db[v];
        }
        store_col4(a.dz2T, a.R, r0w, 16 * n + i16, kg, db);
        dw3p[n] = s3;
        db2p[n] = s2;
    }
    wave_lds_sync();

    // ---- dgrad of layer 2: dh1 = dz2 W2^T, then through GELU
    float db1p[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&act[wid][i16][32 * s + 8 * kg]));
            const bf16x8 b = load_bf16x8(a.W2 + (16 * n + i16) * kH + 32 * s + 8 * kg);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, acc, 0, 0, 0);
        }
        float s1 = 0.f;
        bf16_t db[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float d = acc[v] * gp1[n][v];
            s1 += d;
            db[v] = to_bf16(d);
        }
        store_col4(a.dz1T, a.R, r0w, 16 * n + i16, kg, db);
        db1p[n] = s1;
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---- per-wave sums over its 16 rows (the 4 row groups kg), then per block
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        for (int off = 16; off < 64; off <<= 1) {
            dw3p[n] += __shfl_xor(dw3p[n], off);
            db2p[n] += __shfl_xor(db2p[n], off);
            db1p[n] += __shfl_xor(db1p[n], off);
        }
    }
    // db3 and the loss are per row group (lanes of one kg hold identical values)
    for (int off = 16; off < 64; off <<= 1) {
        db3 += __shfl_xor(db3, off);
        lossp += __shfl_xor(lossp, off);
    }
    if (kg == 0) {
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            part[wid][16 * n + i16] = db1p[n];
            part[wid][kH + 16 * n + i16] = db2p[n];
            part[wid][2 * kH + 16 * n + i16] = dw3p[n];
        }
        if (i16 == 0) {
            part[wid][3 * kH] = db3;
            part[wid][3 * kH + 1] = lossp;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kPart; k += 256)
        a.part[(int64_t)blockIdx.x * kPart + k] = ((part[0][k] + part[1][k]) + part[2][k]) + part[3][k];
}

// dW (M x 128) = L Rt^T over a chunk of the step's K rows: L is [M][K], Rt
// is [128][K] (bf16, the transposed activations / deltas).  blockIdx.x = 0:
// dW2 (M = 128: L = h1^T, Rt = dz2^T), 1: dW1 (M = 32: L = X^T, Rt = dz1^T);
// blockIdx.y = ks covers rows [ks Kc, (ks + 1) Kc).  Each wave owns one
// output sub-tile (dW2: 64 x 64, waves in a 2 x 2 grid; dW1: 32 x 32, waves
// side by side) over the whole chunk, so every L and Rt element of the chunk
// is read once per workgroup; the partial tile goes to wpart[ks][W1 | b1
// gap | W2] and the update kernel sums the ks partials in a fixed order.
template <int TI, int TJ>
__device__ inline void wgrad_tile(const bf16_t* L, const bf16_t* Rt, int64_t K, int kb0, int kb1, int r0, int c0,
                                  float* out, int lane)
{
    const int i16 = lane & 15, kg = lane >> 4;
    f32x4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16_t* La[TI];
    const bf16_t* Rb[TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i) La[i] = L + (int64_t)(r0 + 16 * i + i16) * K + 8 * kg;
#pragma unroll
    for (int j = 0; j < TJ; ++j) Rb[j] = Rt + (int64_t)(c0 + 16 * j + i16) * K + 8 * kg;
    // the next k step's fragments are loaded while this one's MFMAs run
    bf16x8 av[TI], bv[TJ];
    if (kb0 < kb1) {
#pragma unroll
        for (int i = 0; i < TI; ++i) av[i] = load_bf16x8(La[i] + kb0);
#pragma unroll
        for (int j = 0; j < TJ; ++j) bv[j] = load_bf16x8(Rb[j] + kb0);
    }
    for (int kb = kb0; kb < kb1; kb += 32) {
        bf16x8 an[TI], bn[TJ];
        const int kn = kb + 32 < kb1 ? kb + 32 : kb;
#pragma unroll
        for (int i = 0; i < TI; ++i) an[i] = load_bf16x8(La[i] + kn);
#pragma unroll
        for (int j = 0; j < TJ; ++j) bn[j] = load_bf16x8(Rb[j] + kn);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TI; ++i) av[i] = an[i];
#pragma unroll
        for (int j = 0; j < TJ; ++j) bv[j] = bn[j];
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) out[(r0 + 16 * i + 4 * kg + v) * kH + c0 + 16 * j + i16] = acc[i][j][v];
}

// blockIdx.x = 2: the forward/backward workgroups' partial sums (biases,
// w3, b3, loss) of blocks [ks bc, (ks + 1) bc), summed in order, into the
// row's block-sum slots.
__global__ __launch_bounds__(256) void k_mlp_wgrad(const bf16_t* XT, const bf16_t* dz1T, const bf16_t* h1T,
                                                   const bf16_t* dz2T, int32_t K, int32_t Kc, const float* part,
                                                   int32_t blocks, int32_t bc, float* wpart)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int ks = blockIdx.y;
    const int kb0 = ks * Kc, kb1 = min(K, (ks + 1) * Kc);   // Kc and K: multiples of 32
    float* out = wpart + (int64_t)ks * kWRow;
    if (blockIdx.x == 0) {
        wgrad_tile<4, 4>(h1T, dz2T, K, kb0, kb1, 64 * (wid >> 1), 64 * (wid & 1), out + oW2, lane);
    } else if (blockIdx.x == 1) {
        wgrad_tile<2, 2>(XT, dz1T, K, kb0, kb1, 0, 32 * wid, out + oW1, lane);
    } else {
        const int b0 = ks * bc, b1 = min(blocks, (ks + 1) * bc);
        for (int k = threadIdx.x; k < kPart; k += 256) {
            float s = 0.f;
            for (int b = b0; b < b1; ++b) s += part[(int64_t)b * kPart + k];
            out[ob2 + k] = s;
        }
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

// Gradient assembly and Adam: 64 parameters per workgroup, sixteen threads
// per parameter, thread q summing the partial rows q, q + 16, ... in eight
// interleaved running sums joined in a fixed order, the sixteen sums then
// added in a fixed order.  Index kParams is the loss.
constexpr int kUpdSlices = 16;

__device__ inline float strided_sum(const float* base, int64_t stride, int count, int q)
{
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int k = q, j = 0;
    for (; k + 7 * kUpdSlices < count; k += 8 * kUpdSlices)
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] += base[(int64_t)(k + t * kUpdSlices) * stride];
    for (; k < count; k += kUpdSlices, ++j) acc[j & 7] += base[(int64_t)k * stride];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

__global__ __launch_bounds__(1024) void k_mlp_update(const UpdateArgs u)
{
    __shared__ float red[kUpdSlices][64];
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + c;
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
    float* wpart = nullptr;  // [ks][ob2]
    int64_t* idx = nullptr;
    bf16_t* XT = nullptr;
    bf16_t* h1T = nullptr;
    bf16_t* dz2T = nullptr;
    bf16_t* dz1T = nullptr;
    float* part = nullptr;
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

#ifndef MCINV_MLP_WGRAD_ROWS
#define MCINV_MLP_WGRAD_ROWS 256
#endif
// Row splits of the weight-gradient GEMMs: about MCINV_MLP_WGRAD_ROWS rows
// each, at most 512.
int32_t ks_of(int32_t R) { return std::max(1, std::min(512, R / MCINV_MLP_WGRAD_ROWS)); }
int32_t kc_of(int32_t R)
{
    const int32_t ks = ks_of(R);
    return ((R + ks - 1) / ks + 31) / 32 * 32;
}

mcinv_status ensure_step(mcinv_mlp* m, int32_t R)
{
    if (R <= m->Rcap) return MCINV_OK;
    m->Rcap = 0;   // until every buffer below is allocated again
    mfree(m->idx);
    mfree(m->XT);
    mfree(m->h1T);
    mfree(m->dz2T);
    mfree(m->dz1T);
    mfree(m->part);
    mfree(m->wpart);
    MHIP(m, hipMalloc((void**)&m->idx, sizeof(int64_t) * R));
    MHIP(m, hipMalloc((void**)&m->wpart, sizeof(float) * kWRow * (size_t)ks_of(R)));
    MHIP(m, hipMalloc((void**)&m->XT, sizeof(bf16_t) * kF * (size_t)R));
    MHIP(m, hipMalloc((void**)&m->h1T, sizeof(bf16_t) * kH * (size_t)R));
    MHIP(m, hipMalloc((void**)&m->dz2T, sizeof(bf16_t) * kH * (size_t)R));
    MHIP(m, hipMalloc((void**)&m->dz1T, sizeof(bf16_t) * kH * (size_t)R));
    MHIP(m, hipMalloc((void**)&m->part, sizeof(float) * kPart * (size_t)((R + 63) / 64)));
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

// One forward/backward over R rows and the gradient assembly; with `apply`,
// the Adam step.  The rows: drawn from Philox (key = seed, counter word 1 =
// the step about to be taken) with `draw`, else the list in m->idx.
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
    a.XT = m->XT;
    a.h1T = m->h1T;
    a.dz2T = m->dz2T;
    a.dz1T = m->dz1T;
    a.part = m->part;
    a.inv_denom = 1.0f / (float)R;
    const int blocks = R / 64;
    k_mlp_fwd_bwd<true><<<dim3(blocks), dim3(256), 0, m->stream>>>(a);
    MHIP(m, hipGetLastError());
    const int32_t kc = kc_of(R), nks = (R + kc - 1) / kc, bc = (blocks + nks - 1) / nks;
    k_mlp_wgrad<<<dim3(3, nks), dim3(256), 0, m->stream>>>(m->XT, m->dz1T, m->h1T, m->dz2T, R, kc, m->part, blocks,
                                                          bc, m->wpart);
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
    k_mlp_update<<<dim3((kParams + 1 + 63) / 64), dim3(64 * kUpdSlices), 0, m->stream>>>(u);
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
        k_mlp_fwd_bwd<false><<<dim3((unsigned)((a.R + 63) / 64)), dim3(256), 0, m->stream>>>(a);
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
    if (hipMalloc((void**)&m->P, sizeof(float) * kParams) != hipSuccess ||
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
    mfree(m->XT);
    mfree(m->h1T);
    mfree(m->dz2T);
    mfree(m->dz1T);
    mfree(m->part);
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
