// Kernel argument blocks and launchers of the mcinv device code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace mcinv {

// One colour launch of the sweep (eqs 4 and 5) over positions
// [row_begin, row_end), all pair tiles.
template <typename V>
struct SweepArgs {
    const RowRec* rows;
    const Entry<V>* ent;
    const Scales<V>* sc;
    V* z;                    // state [n][ld], positions x pairs
    V* w;
    int64_t ld;              // padded pairs per state row (multiple of 4)
    int64_t P;               // real pairs (pairs >= P are padding)
    int64_t row_begin, row_end;
    int64_t tile0;           // first pair tile of this launch (blockIdx.y offset)
    int64_t n;               // rows (positions) of the matrix
    uint32_t key0, key1;     // Philox key = seed
    uint32_t sweep;          // Philox counter word 1
    uint32_t stream;         // Philox counter word 3
    uint32_t pair_block0;    // global index of this context's first pair / 4 (Philox counter word 2 offset)
    int32_t noise;           // NoiseKind
    int32_t lg_shift;        // log2(lanes summed into one diagonal column)
    double* diag;            // slot accumulator [tiles][n][64 >> lg_shift] (x2 complex) or null
    double* tpart;           // per-workgroup trace partials of this launch, or null
    int32_t* flag;           // divergence flag (bit 0)
    typename Real<V>::type thresh;
    int32_t xcd_order;       // 0: natural workgroup order; 1: contiguous tile ranges per XCD;
                             // 2: runs of 16 consecutive row blocks per XCD; 3: pair tiles fastest
    int32_t nt_stores;       // nonzero: store new state rows non-temporally
};

// Launch over pair tiles [a.tile0, a.tile0 + ntiles).  herm: C is hermitian
// with a positive diagonal and only z is swept (w = z, eq 2).
template <typename V>
hipError_t launch_sweep(const SweepArgs<V>& a, int64_t ntiles, bool sample, bool herm, hipStream_t stream);

hipError_t launch_noise_values(bool fp64, uint64_t seed, uint32_t stream_id, int32_t kind, int64_t count,
                               const int64_t* row, const int64_t* sweep, const int64_t* pair, double* out,
                               hipStream_t stream);

}  // namespace mcinv
