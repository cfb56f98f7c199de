// Dense requested-block moments on the matrix cores (eq 1/C), precision form.
//
// For each chain group g and sample:  B[g][r][t] += sum_{p in g} z[I_r][p] w[J_t][p]
// with fp32 state, as bf16x3 split products (mfma_tile.h) accumulated in fp32
// over the group's pairs, then added to the fp64 sums.
//
// Both operands are "row = output index, contiguous along pairs": lane l of a
// 16x16x32 MFMA holds row (l mod 16), pairs 8*(l div 16) .. +7, so each lane
// reads its 8 fp32 values straight from the state with two 16-byte loads.
// A wave owns a 32 x 32 output tile (2 x 2 MFMA tiles) of one group; a
// workgroup holds four groups of the same tile.
#include "device_common.h"
#include "mfma_tile.h"
#include "moments.h"
#include "sweep.h"

namespace mcinv {

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
    bf16x3_tile(zrow, zok, wrow, wok, pbeg, pend, kg, acc);

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
