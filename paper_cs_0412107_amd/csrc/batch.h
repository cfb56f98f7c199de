// Batched form: many matrices and their chains in one persistent launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace mcinv {

// One work item of a sweep: rows [row_begin, row_end) (global positions) of one
// colour of matrix m, or (kind 1) the block moments of matrix m.
struct BItem {
    int32_t m;
    int32_t kind;
    int64_t row_begin;
    int64_t row_end;
    int32_t prior;      // items of matrix m in earlier phases of the same sweep
    int32_t pad;
};

struct BMat {
    int64_t row0;            // first global position of the matrix
    int64_t n;
    int32_t items_per_sweep;  // work items of this matrix in one sweep
    uint32_t stream;          // Philox counter word 3
    int64_t blk;              // offset of its block index lists, or -1
};

// Device-resident progress of the batch; the last workgroup of a launch
// advances it and clears the queue and completion counters.
struct BatchClock {
    int64_t sweep;       // absolute index of the next sweep (Philox counter word 1)
    int64_t sample;      // samples accumulated so far
    uint32_t queue;      // next work item to hand out
    uint32_t exited;     // workgroups that have finished this launch
    int32_t error;       // set when a dependency wait exceeded its bound
    int32_t pad;
};

struct BatchArgs {
    const RowRec* rows;          // global positions; begin = global entry offset
    const Entry<float>* ent;     // col = global position
    const Scales<float>* sc;
    float* z;                    // [rows][P]
    float* w;
    int32_t P;                   // pairs per matrix (16, 32, 64, 128 or 256)
    int32_t lane_shift;          // log2(lanes per row) = log2(P / 4)
    const BItem* items;          // one sweep's items in (colour, matrix, chunk) order
    int64_t items_per_sweep;
    int64_t nsweeps;             // sweeps in this launch
    int32_t sample;              // accumulate moments
    int32_t grab;                // items taken per queue access
    const BMat* mats;
    int32_t nmats;
    uint32_t* done;              // per matrix: items completed in this launch
    BatchClock* clock;
    uint32_t key0, key1;
    int32_t noise;
    uint32_t spin_limit;         // bound on one dependency wait (polls)
    // moments
    int32_t G;                   // groups per matrix (P % G == 0, P/G >= 4)
    int32_t nslots_diag;         // time batches of the diagonal accumulator (1: groups only)
    int32_t nslots_block;        // time batches of the block accumulator
    int32_t pad_;
    int64_t batch_len;           // samples per time batch
    int64_t nrows;               // total rows of the batch
    double* diag;                // [slots][nrows][G] or null
    int32_t bdim;                // requested block edge per matrix (<= 128), 0 = none
    const int64_t* bI;           // [nmats][bdim] global positions of block rows
    const int64_t* bJ;
    double* block;               // [slots][nmats][bdim][bdim] or null
    int32_t* flag;               // divergence flag
    float thresh;
};

hipError_t launch_batch(const BatchArgs& a, int grid, hipStream_t stream);
// Phased schedule: the items of one phase, one workgroup each.
hipError_t launch_batch_phase(const BatchArgs& a, const BItem* items, int64_t nitems, bool block_phase,
                              hipStream_t stream);
hipError_t launch_batch_tick(BatchClock* clock, bool sample, hipStream_t stream);
// out[row_mat[q]] = max |x[q * ld]| (double bits, atomic max; clear out first).
hipError_t launch_batch_max_abs(const float* x, int64_t nrows, int32_t ld, const int32_t* row_mat,
                                unsigned long long* out, hipStream_t stream);
int batch_kernel_occupancy();  // workgroups per CU the batch kernel can keep resident

}  // namespace mcinv
