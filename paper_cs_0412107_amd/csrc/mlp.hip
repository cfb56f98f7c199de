// The learned surrogate's network: MLP 32 -> 128 -> 128 -> 1 with GELU
// (erf form), bf16 operands on the matrix cores with fp32 accumulation, fp32
// master weights and Adam (Kingma & Ba, 2015).  It predicts y_i = c_ii
// (C^-1)_ii from the 32 local features of row i.
//
// Kernels
//   k_mlp_fwd_bwd : one wave = 16 rows.  Layer 1 and 2 products on
//                   v_mfma_f32_16x16x32_bf16 (A = activations, B = weights
//                   from global), GELU in fp32, output layer in fp32.  With
//                   `backward`: the weighted-MSE gradient flows back through
//                   layer 3 (fp32), layer 2 (dgrad on MFMA) and both GELUs;
//                   activations and deltas go out transposed as bf16 for the
//                   weight gradients, bias / w3 partial sums per workgroup.
//   k_mlp_wgrad   : dW1 = X^T dz1, dW2 = h1^T dz2 over the step's rows
//                   (32 x 32 tile per workgroup, the rows split over
//                   workgroups and over its 4 waves, summed in a fixed order).
//   k_mlp_update  : gradient assembly (partials summed in a fixed order),
//                   Adam step, bf16 copies of the weights.
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

typedef unsigned short bf16_t;

__device__ inline bf16_t to_bf16(float x) { return bf16_rne(x); }

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
    int32_t R;               // rows of this call
    int32_t backward;
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

__global__ __launch_bounds__(256) void k_mlp_fwd_bwd(const MlpArgs a)
{
    // act: h1 (bf16) as layer 2's A operand, then dz2 (bf16) as the dgrad A
    // operand; gp1: gelu'(z1) kept from the forward pass for the backward
    // one, so no first-layer pre-activations stay in registers.
    __shared__ __align__(16) bf16_t act[4][16][kActLd];
    __shared__ __align__(16) bf16_t dz1s[4][16][kActLd];
    __shared__ float gp1[4][16][kH + 4];
    __shared__ float part[4][kPart];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int i16 = lane & 15, kg = lane >> 4;
    const int64_t r0w = (int64_t)blockIdx.x * 64 + wid * 16;
    auto row_of = [&](int64_t r) { return a.idx ? a.idx[r] : a.row0 + r; };
    const float* P = a.P;
    constexpr float kRs2 = 0.70710678118654752f, kRs2pi = 0.39894228040143268f;

    // ---- layer 1: A = normalised features (row i16, features 8kg..8kg+7)
    const int64_t ra = r0w + i16;
    const bool aok = ra < a.R;
    bf16x8 a1;
    {
        unsigned short u[8];
        const float* x = a.X + (aok ? row_of(ra) : 0) * kF + 8 * kg;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float xn = aok ? (x[e] - a.mean[8 * kg + e]) * a.inv_std[8 * kg + e] : 0.0f;
            u[e] = to_bf16(xn);
            if (a.backward) act[wid][i16][8 * kg + e] = u[e];
        }
        u16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = u[e];
        a1 = __builtin_bit_cast(bf16x8, v);
    }
    if (a.backward) {   // backward launches cover whole 64-row blocks
        __syncthreads();
        store_transposed(act[wid], kF, a.XT, a.R, r0w, lane);
        __syncthreads();
    }
    // z1 -> h1 = GELU(z1) into LDS (bf16) and h1^T; gelu'(z1) into LDS
    for (int n = 0; n < 8; ++n) {
        const bf16x8 b = load_bf16x8(a.W1T + (16 * n + i16) * kF + 8 * kg);
        const f32x4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        const float bias = P[ob1 + 16 * n + i16];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float zz = z[v] + bias;
            const float e = erff(zz * kRs2);
            const bf16_t hb = to_bf16(0.5f * zz * (1.0f + e));
            act[wid][4 * kg + v][16 * n + i16] = hb;
            if (a.backward)
                gp1[wid][4 * kg + v][16 * n + i16] = 0.5f * (1.0f + e) + zz * expf(-0.5f * zz * zz) * kRs2pi;
        }
    }
    __syncthreads();
    if (a.backward) store_transposed(act[wid], kH, a.h1T, a.R, r0w, lane);

    // ---- layer 2
    f32x4 z2[8];
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
#pragma unroll
        for (int v = 0; v < 4; ++v) z2[n][v] = acc[v] + bias;
        // one column block at a time: hoisting every block's weight loads
        // measured 1.4x slower (register pressure, two waves per SIMD)
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---- layer 3 (fp32): out_v for rows r0w + 4kg + v
    float out[4] = {0.f, 0.f, 0.f, 0.f};
    for (int n = 0; n < 8; ++n) {
        const float w3 = P[ow3 + 16 * n + i16];
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v] += 0.5f * z2[n][v] * (1.0f + erff(z2[n][v] * kRs2)) * w3;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        for (int off = 1; off < 16; off <<= 1) out[v] += __shfl_xor(out[v], off);
        out[v] += P[ob3];
    }
    if (!a.backward) {
        if (i16 == 0)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t rd = r0w + 4 * kg + v;
                if (rd < a.R) a.out[rd] = out[v];
            }
        return;
    }

    // ---- loss gradient
    float dout[4], lossp = 0.f, db3 = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t rd = r0w + 4 * kg + v;
        float dv = 0.f;
        if (rd < a.R) {
            const int64_t row = row_of(rd);
            const float diff = out[v] - a.y[row];
            dv = 2.0f * a.w[row] * diff * a.inv_denom;
            lossp += a.w[row] * diff * diff * a.inv_denom;
        }
        dout[v] = dv;
        db3 += dv;
    }

    // ---- layer 3 backward and layer 2 deltas, written straight to LDS (bf16)
    float dw3p[8], db2p[8];
    __syncthreads();  // every wave is done reading h1 from LDS
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const float w3 = P[ow3 + 16 * n + i16];
        float s3 = 0.f, s2 = 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float zz = z2[n][v];
            const float e = erff(zz * kRs2);
            s3 += 0.5f * zz * (1.0f + e) * dout[v];
            const float d = dout[v] * w3 * (0.5f * (1.0f + e) + zz * expf(-0.5f * zz * zz) * kRs2pi);
            s2 += d;
            act[wid][4 * kg + v][16 * n + i16] = to_bf16(d);
        }
        dw3p[n] = s3;
        db2p[n] = s2;
    }
    __syncthreads();
    store_transposed(act[wid], kH, a.dz2T, a.R, r0w, lane);

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
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float d = acc[v] * gp1[wid][4 * kg + v][16 * n + i16];
            s1 += d;
            dz1s[wid][4 * kg + v][16 * n + i16] = to_bf16(d);
        }
        db1p[n] = s1;
        __builtin_amdgcn_sched_barrier(0);
    }

    __syncthreads();
    store_transposed(dz1s[wid], kH, a.dz1T, a.R, r0w, lane);

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

// dW (rows x 128) = L Rt^T over K training rows: L is [rows][K], Rt is
// [128][K] (bf16, the transposed activations / deltas).  Workgroup (tile,
// ks) covers the rows [ks Kc, (ks + 1) Kc) of the step; its wave `wid` takes
// the 32-row slabs wid, wid + 4, ... of that range and the four partial tiles
// are summed in order.  The ks partials go to wpart[ks][W1 | b1 gap | W2] and
// are summed in order of ks by the update kernel.
__global__ __launch_bounds__(256) void k_mlp_wgrad(const bf16_t* XT, const bf16_t* dz1T, const bf16_t* h1T,
                                                   const bf16_t* dz2T, int32_t K, int32_t Kc, float* wpart)
{
    __shared__ float red[4][32][33];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int i16 = lane & 15, kg = lane >> 4;
    // tiles 0..3: dW1 (32 x 128), tiles 4..19: dW2 (128 x 128)
    const int tile = blockIdx.x;
    const int ks = blockIdx.y;
    const bf16_t *L, *Rt;
    int r0, c0, base;
    if (tile < 4) {
        L = XT; Rt = dz1T; r0 = 0; c0 = 32 * tile; base = oW1;
    } else {
        L = h1T; Rt = dz2T; r0 = 32 * ((tile - 4) / 4); c0 = 32 * ((tile - 4) % 4); base = oW2;
    }
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int k_end = min(K, (ks + 1) * Kc);   // Kc and K: multiples of 32
    for (int kb = ks * Kc + 32 * wid; kb < k_end; kb += 128) {
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            av[t] = load_bf16x8(L + (int64_t)(r0 + 16 * t + i16) * K + kb + 8 * kg);
            bv[t] = load_bf16x8(Rt + (int64_t)(c0 + 16 * t + i16) * K + kb + 8 * kg);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[wid][16 * i + 4 * kg + v][16 * j + i16] = acc[i][j][v];
    __syncthreads();
    float* out = wpart + (int64_t)ks * ob2;
    for (int t = threadIdx.x; t < 32 * 32; t += 256) {
        const int r = t / 32, c = t % 32;
        const float s = ((red[0][r][c] + red[1][r][c]) + red[2][r][c]) + red[3][r][c];
        out[base + (r0 + r) * kH + c0 + c] = s;
    }
}

// psum[k] = sum over the forward/backward workgroups of part[b][k]: one
// wave per k, lane l summing b = l, l + 64, ... in order, then a fixed
// butterfly across the lanes.
__global__ __launch_bounds__(64) void k_mlp_reduce_parts(const float* part, int32_t blocks, float* psum)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    float v = 0.f;
    for (int b = lane; b < blocks; b += 64) v += part[(int64_t)b * kPart + k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) psum[k] = v;
}

struct UpdateArgs {
    float* P;                // master parameters
    float* m;                // Adam first moments
    float* v;                // Adam second moments
    float* grads;            // the assembled gradient [kParams]
    const float* wpart;      // weight-gradient partials [nks][ob2]
    int32_t nks;
    const float* psum;       // [kPart] summed workgroup partials
    int32_t apply;           // 0: only assemble the gradient
    float lr, beta1, beta2, eps;
    float bc1, bc2;          // 1 - beta^t
    bf16_t* W1T;
    bf16_t* W2T;
    bf16_t* W2;
    float* loss_out;         // loss of this step, or null
};

__global__ __launch_bounds__(256) void k_mlp_update(const UpdateArgs u)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && u.loss_out) *u.loss_out = u.psum[3 * kH + 1];
    if (p >= kParams) return;
    float g;
    if ((p >= oW1 && p < ob1) || (p >= oW2 && p < ob2)) {
        g = 0.f;
        for (int k = 0; k < u.nks; ++k) g += u.wpart[(int64_t)k * ob2 + p];
        u.grads[p] = g;
    } else {
        int k;
        if (p < oW2)
            k = p - ob1;               // db1
        else if (p < ow3)
            k = kH + (p - ob2);        // db2
        else if (p < ob3)
            k = 2 * kH + (p - ow3);    // dw3
        else
            k = 3 * kH;                // db3
        g = u.psum[k];
        u.grads[p] = g;
    }
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

// Philox-drawn rows of one training step: idx[r] = floor(u * N).
__global__ __launch_bounds__(256) void k_mlp_sample_rows(uint32_t k0, uint32_t k1, uint32_t step, int64_t N,
                                                         int32_t R, int64_t* idx)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    uint32_t c0 = (uint32_t)r, c1 = step, c2 = 0x5EEDu, c3 = 0xA11CEu;
    Philox::block(c0, c1, c2, c3, k0, k1);
    const uint64_t x = ((uint64_t)c0 << 32) | c1;
    idx[r] = (int64_t)(((unsigned __int128)x * (uint64_t)N) >> 64);
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
    float* psum = nullptr;   // [kPart]
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

// Row splits of the weight-gradient GEMMs: about 512 rows each, at most 64.
int32_t ks_of(int32_t R) { return std::max(1, std::min(64, R / 512)); }
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
    MHIP(m, hipMalloc((void**)&m->wpart, sizeof(float) * ob2 * (size_t)ks_of(R)));
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

// One forward/backward over R rows (idx on device) and the gradient assembly;
// with `apply`, the Adam step.
mcinv_status run_step(mcinv_mlp* m, int32_t R, bool apply, float lr, float* loss_dev)
{
    MlpArgs a = base_args(m);
    a.X = m->X;
    a.y = m->y;
    a.w = m->w;
    a.idx = m->idx;
    a.R = R;
    a.backward = 1;
    a.XT = m->XT;
    a.h1T = m->h1T;
    a.dz2T = m->dz2T;
    a.dz1T = m->dz1T;
    a.part = m->part;
    a.inv_denom = 1.0f / (float)R;
    const int blocks = R / 64;
    k_mlp_fwd_bwd<<<dim3(blocks), dim3(256), 0, m->stream>>>(a);
    MHIP(m, hipGetLastError());
    const int32_t kc = kc_of(R), nks = (R + kc - 1) / kc;
    k_mlp_wgrad<<<dim3(20, nks), dim3(256), 0, m->stream>>>(m->XT, m->dz1T, m->h1T, m->dz2T, R, kc, m->wpart);
    MHIP(m, hipGetLastError());
    UpdateArgs u{};
    u.P = m->P;
    u.m = m->m;
    u.v = m->v;
    u.grads = m->grads;
    u.wpart = m->wpart;
    u.nks = nks;
    k_mlp_reduce_parts<<<dim3(kPart), dim3(64), 0, m->stream>>>(m->part, blocks, m->psum);
    MHIP(m, hipGetLastError());
    u.psum = m->psum;
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
    k_mlp_update<<<dim3((kParams + 255) / 256), dim3(256), 0, m->stream>>>(u);
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
        a.backward = 0;
        a.out = dout + r0;
        k_mlp_fwd_bwd<<<dim3((unsigned)((a.R + 63) / 64)), dim3(256), 0, m->stream>>>(a);
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
        hipMalloc((void**)&m->loss, sizeof(float) * 1) != hipSuccess ||
        hipMalloc((void**)&m->psum, sizeof(float) * kPart) != hipSuccess)
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
    mfree(m->psum);
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
        k_mlp_sample_rows<<<dim3((batch_rows + 255) / 256), dim3(256), 0, m->stream>>>(
            (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), (uint32_t)(m->t + 1), m->N, batch_rows, m->idx);
        MHIP(m, hipGetLastError());
        const mcinv_status st = run_step(m, batch_rows, true, lr, dloss.p ? dloss.p + s : nullptr);
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
