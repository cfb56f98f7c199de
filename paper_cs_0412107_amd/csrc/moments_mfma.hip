// Dense requested-block moments on the matrix cores (eq 1/C), precision form.
//
// For each chain group g and sample:  B[g][r][t] += sum_{p in g} z[I_r][p] w[J_t][p]
// with fp32 state.  Every fp32 value x is split into bf16 hi = rne(x) and
// lo = rne(x - hi); the product is hi*hi' + hi*lo' + lo*hi' (the lo*lo' term,
// ~2^-16 relative, is dropped), each on v_mfma_f32_16x16x32_bf16 with fp32
// accumulation over the group's pairs, then added to the fp64 sums.
//
// Both operands are "row = output index, contiguous along pairs": lane l of a
// 16x16x32 MFMA holds row (l mod 16), pairs 8*(l div 16) .. +7, so each lane
// reads its 8 fp32 values straight from the state with two 16-byte loads.
// A wave owns a 32 x 32 output tile (2 x 2 MFMA tiles) of one group; a
// workgroup holds four groups of the same tile.
#include "device_common.h"
#include "sweep.h"

namespace mcinv {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ inline void split8(const float v[8], bf16x8& hi, bf16x8& lo)
{
    u16x8 h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const unsigned short hb = bf16_rne(v[e]);
        const float hf = __uint_as_float((uint32_t)hb << 16);
        h[e] = hb;
        l[e] = bf16_rne(v[e] - hf);
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

__device__ inline void load8(const float* row, int64_t p, int64_t pend, bool valid, float v[8])
{
    if (valid && p + 7 < pend) {
        const float4 x0 = *reinterpret_cast<const float4*>(row + p);
        const float4 x1 = *reinterpret_cast<const float4*>(row + p + 4);
        v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
        v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (valid && p + e < pend) ? row[p + e] : 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_block_bf16x3(const BlockArgs<float> a)
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.z * 4 + wid;
    if (g >= a.G) return;
    const int64_t r0 = (int64_t)blockIdx.y * 32, t0 = (int64_t)blockIdx.x * 32;
    const int64_t pbeg = g * a.gs, pend = pbeg + a.gs;
    const int i16 = lane & 15, kg = lane >> 4;

    const float* zrow[2];
    const float* wrow[2];
    bool zok[2], wok[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int64_t r = r0 + 16 * t + i16, c = t0 + 16 * t + i16;
        zok[t] = r < a.nI;
        wok[t] = c < a.nJ;
        zrow[t] = a.z + (zok[t] ? a.I[r] : 0) * a.ld;
        wrow[t] = a.w + (wok[t] ? a.J[c] : 0) * a.ld;
    }

    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int64_t kb = pbeg; kb < pend; kb += 32) {
        const int64_t p = kb + 8 * kg;
        bf16x8 zh[2], zl[2], wh[2], wl[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            float v[8];
            load8(zrow[t], p, pend, zok[t], v);
            split8(v, zh[t], zl[t]);
            load8(wrow[t], p, pend, wok[t], v);
            split8(v, wh[t], wl[t]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh[i], wh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh[i], wl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zl[i], wh[j], acc[i][j], 0, 0, 0);
            }
    }

    // Output layout of a 16x16 MFMA tile: lane l holds rows 4*(l div 16) + v,
    // column l mod 16.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t c = t0 + 16 * j + i16;
            if (c >= a.nJ) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = r0 + 16 * i + 4 * kg + v;
                if (r < a.nI) a.acc[(g * a.nI + r) * a.nJ + c] += (double)acc[i][j][v];
            }
        }
}

hipError_t launch_block_bf16x3(const BlockArgs<float>& a, hipStream_t stream)
{
    if (a.nI <= 0 || a.nJ <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.nJ + 31) / 32), (unsigned)((a.nI + 31) / 32), (unsigned)((a.G + 3) / 4));
    k_block_bf16x3<<<grid, dim3(256), 0, stream>>>(a);
    return hipGetLastError();
}

}  // namespace mcinv
