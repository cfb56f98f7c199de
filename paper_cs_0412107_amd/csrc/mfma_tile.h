// bf16x3 split products on the gfx950 matrix cores (shared by the single-matrix
// block-moment kernel and the batched form).
//
// Every fp32 value x is split into bf16 hi = rne(x) and lo = rne(x - hi); the
// product of two values is hi*hi' + hi*lo' + lo*hi' (lo*lo', ~2^-16 relative,
// is dropped), accumulated in fp32 by v_mfma_f32_16x16x32_bf16.
//
// Operand layout: lane l of a 16x16x32 MFMA holds row (l mod 16) and the 8
// consecutive k values 8*(l div 16) .. +7; the 16x16 fp32 result holds rows
// 4*(l div 16) + v, column l mod 16, in its four registers v = 0..3.
#pragma once

#include "device_common.h"

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

// v[0..7] = row[p .. p+7] (zero beyond pend or when !valid); two 16-byte loads
// when the whole run is in range (row + p is 16-byte aligned by construction).
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

// acc[i][j] += Z W^T over pairs [pbeg, pend) for the 32 x 32 tile whose
// rows are zrow[0..1] (rows i16 and 16+i16 of the tile, for this lane) and
// columns wrow[0..1].
__device__ inline void bf16x3_tile(const float* const zrow[2], const bool zok[2], const float* const wrow[2],
                                   const bool wok[2], int64_t pbeg, int64_t pend, int kg, f32x4 acc[2][2])
{
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
}

// acc += Z W^T over pairs [pbeg, pend) for one 16 x 16 tile: this lane holds
// row zrow (tile row l mod 16) and column row wrow.  Same MFMA sequence per
// output tile as bf16x3_tile, in a quarter of the registers.
__device__ inline void bf16x3_tile16(const float* zrow, bool zok, const float* wrow, bool wok, int64_t pbeg,
                                     int64_t pend, int kg, f32x4& acc)
{
    for (int64_t kb = pbeg; kb < pend; kb += 32) {
        const int64_t p = kb + 8 * kg;
        bf16x8 zh, zl, wh, wl;
        float v[8];
        load8(zrow, p, pend, zok, v);
        split8(v, zh, zl);
        load8(wrow, p, pend, wok, v);
        split8(v, wh, wl);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh, wh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh, wl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zl, wh, acc, 0, 0, 0);
    }
}

}  // namespace mcinv
