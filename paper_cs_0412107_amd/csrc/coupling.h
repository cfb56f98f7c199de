// Noiseless difference iteration of two coupled paths (Sec. 2.3, eq 12).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace mcinv {

// One colour [row_begin, row_end) of dz_i <- -sum_j u_ij dz_j and (unless
// herm) dw_i <- -sum_j v_ij dw_j; dz, dw hold one value per position.
template <typename V>
hipError_t launch_coupling_sweep(const RowRec* rows, const Entry<V>* ent, int64_t row_begin, int64_t row_end,
                                 bool herm, V* dz, V* dw, hipStream_t stream);

}  // namespace mcinv
