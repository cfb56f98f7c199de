// Internal steps of the surrogate shared by its entry points (features.hip,
// mlp.hip, gate.hip): features left in device memory, the network run on
// device rows, and the gate's decision from two feature columns.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mcinv.h"

namespace mcinv {

// Features of a real CSR matrix (validated here) computed on `device`:
// *d_features receives [n][MCINV_N_FEATURES] floats in device memory that the
// caller releases with hipFree.  Returns a status; on failure *err says why.
// diag (may be NULL) receives c_ii per row (host).
mcinv_status features_on_device(int32_t device, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                const int32_t* col_idx, const double* values, float** d_features, std::string* err,
                                std::vector<double>* diag = nullptr);

// Columns a and b of device features [n][MCINV_N_FEATURES] into host out[n][2].
mcinv_status features_pick_two(const float* d_features, int64_t n, int32_t a, int32_t b, float* out,
                               std::string* err);

// The network on device rows dX[N][MCINV_N_FEATURES] into device dout[N]
// (on the network's stream, which is synchronised before returning).
mcinv_status mlp_predict_device(mcinv_mlp* m, const float* dX, int64_t N, float* dout, std::string* err);

// The gate's fallback flag of each of N rows whose binning features sit at
// columns ca and cb of host rows of ld floats.
void gate_fallback_rows(const mcinv_gate* g, int64_t N, const float* X, int64_t ld, int32_t ca, int32_t cb,
                        uint8_t* fallback);
int32_t gate_feature_a(const mcinv_gate* g);
int32_t gate_feature_b(const mcinv_gate* g);

}  // namespace mcinv
