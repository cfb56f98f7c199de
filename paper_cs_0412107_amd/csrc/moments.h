// Moment accumulation and finalisation kernels: argument blocks and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace mcinv {

// ---------------------------------------------------------------- moments --
// Dense block moments B[g][r][t] += sum_{p in group g} z[I_r][p] conj(w[J_t][p]) (eq 1/C).
template <typename V>
struct BlockArgs {
    const V* z;
    const V* w;
    int64_t ld;
    const int64_t* I;        // positions of the requested rows
    const int64_t* J;        // positions of the requested columns
    int64_t nI, nJ;
    int64_t gs;              // pairs per group
    int64_t G;
    double* acc;             // slot accumulator [G][nI][nJ] (x2 complex)
};

template <typename V>
hipError_t launch_block_fp64(const BlockArgs<V>& a, hipStream_t stream);
hipError_t launch_block_bf16x3(const BlockArgs<float>& a, hipStream_t stream);

// Entry moments E[g][e] += sum_{p in g} z[ei][p] conj(w[ej][p]).
template <typename V>
hipError_t launch_entries(const V* z, const V* w, int64_t ld, const int64_t* ei, const int64_t* ej,
                          int64_t ne, int64_t gs, int64_t G, double* acc, hipStream_t stream);

// acc[m] = acc[2m] + acc[2m+1] for m < half, acc[m] = 0 for half <= m < 2 half.
hipError_t launch_merge_slots(double* acc, int64_t slot_elems, int64_t half, hipStream_t stream);

// Per-sample sum over pairs of w^dagger Q z for a sparse Q in position order
// (CSR qrp[n+1], qcol, qval); partials: ceil(n/4) x pair tiles (x comps).
template <typename V>
struct QTraceArgs {
    const V* z;
    const V* w;
    int64_t ld, P, n;
    const int64_t* qrp;
    const int64_t* qcol;
    const V* qval;
    double* part;
};
// Q rows per wave of the Q-trace kernel; partials: ceil(n / (4 kQRowsPerWave)) per 256-pair tile.
constexpr int kQRowsPerWave = 4;
template <typename V>
hipError_t launch_qtrace(const QTraceArgs<V>& a, hipStream_t stream);

// Largest magnitude of x[q * ld], q < n, into *out (double bits, atomic max;
// clear *out first).
template <typename V>
hipError_t launch_max_abs(const V* x, int64_t n, int64_t ld, unsigned long long* out, hipStream_t stream);

// Deterministic sum of x[count][comps] into out[comps] (two stages, one launch).
hipError_t launch_reduce_sum(const double* x, int64_t count, int comps, double* partial, uint32_t* counter,
                             double* out, hipStream_t stream);

// Cluster finalisation.  Clusters are (slot b, group g); slot b holds
// slot_len[b] samples, each group gs pairs.
struct FinalizeArgs {
    const double* acc;       // diag: [nslots][tiles][n][cpt]; flat: [nslots][G][M]  (x comps)
    int64_t nslots;
    int64_t slot_stride;     // doubles per slot
    const double* slot_len;  // samples per slot
    int64_t G;
    int64_t gs;
    int64_t M;               // values (positions or flat entries)
    int64_t A;               // diag only: columns (tiles x cpt)
    int64_t cpt;             // diag only: columns per pair tile
    int64_t pairs_per_col;   // diag only
    int comps;               // 1 real, 2 complex
    const int64_t* out_index;  // position -> output index (diag; optional for flat)
    int64_t gstride;         // flat only: doubles/comps between groups (0: M)
    int64_t mstride;         // flat only: between consecutive values (0: 1)
    double* est;             // [M][comps] (at out_index)
    double* se;              // [M]
    unsigned long long* max_rel;  // diag / flat, may be null: max se/|est| as bits
    const uint8_t* stop_mask;     // diag only, may be null: rows (output index) that max_rel covers
    const int32_t* val_group;     // groups only, may be null: value -> its own slot lengths at
    int64_t slot_len_stride;      //   slot_len + val_group[v] * slot_len_stride (one matrix of a batch)
    double* rel_out;              // groups only, may be null: per value se/|est| (+inf without estimate)
};
hipError_t launch_finalize_diag(const FinalizeArgs& f, hipStream_t stream);
hipError_t launch_finalize_flat(const FinalizeArgs& f, hipStream_t stream);
// Flat layout [nslots][M][G] (G a power of two <= 64), coalesced.
hipError_t launch_finalize_groups(const FinalizeArgs& f, hipStream_t stream);
// out[s] = max of x[begin[s] .. begin[s+1]), one workgroup per segment.
hipError_t launch_segment_max(const double* x, const int64_t* begin, int64_t nseg, double* out, hipStream_t stream);

// Geyer initial-positive-sequence error of the per-sweep trace series.
// out[0..1] = mean (re, im), out[2] = gamma_0 (var), out[3] = sigma^2, out[4] = N_eff, out[5] = SE.
hipError_t launch_geyer(const double* series, int64_t S, int comps, double scale, double* out,
                        hipStream_t stream);

}  // namespace mcinv
