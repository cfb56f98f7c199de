// Difference of two coupled paths (Sec. 2.3): with the same noise, eq 12
// makes z_2 - z_1 follow the noiseless Gauss-Seidel iteration on C d = 0 and
// w_2 - w_1 the one on C^dagger d = 0.  One colour launch updates every row
// of the colour, one thread per row (the difference is the same for all
// chain pairs, so one value per row suffices):
//     dz_i <- -sum_j u_ij dz_j,   dw_i <- -sum_j v_ij dw_j
// with the merged-entry coefficients of the sweep kernel, accumulated in
// entry order with fused multiply-adds -- the same arithmetic as a noiseless
// sweep of the chains themselves.
#include "coupling.h"

namespace mcinv {

template <typename V>
__global__ __launch_bounds__(256) void k_coupling_sweep(const RowRec* rows, const Entry<V>* ent, int64_t row_begin,
                                                        int64_t row_end, bool herm, V* dz, V* dw)
{
    const int64_t q = row_begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= row_end) return;
    const RowRec rr = rows[q];
    const Entry<V>* e = ent + rr.begin;
    V az = vzero<V>(), aw = vzero<V>();
    for (int32_t t = 0; t < rr.count; ++t) {
        const Entry<V> en = e[t];
        az = mul_add(en.u, dz[en.col], az);
        if (!herm) aw = mul_add(en.v, dw[en.col], aw);
    }
    const V zero = vzero<V>();
    dz[q] = noisy_update(zero, typename Real<V>::type(0), az);
    if (!herm) dw[q] = noisy_update(zero, typename Real<V>::type(0), aw);
}

template <typename V>
hipError_t launch_coupling_sweep(const RowRec* rows, const Entry<V>* ent, int64_t row_begin, int64_t row_end,
                                 bool herm, V* dz, V* dw, hipStream_t stream)
{
    const int64_t n = row_end - row_begin;
    if (n <= 0) return hipSuccess;
    k_coupling_sweep<V><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream>>>(rows, ent, row_begin, row_end,
                                                                                    herm, dz, dw);
    return hipGetLastError();
}

template hipError_t launch_coupling_sweep<float>(const RowRec*, const Entry<float>*, int64_t, int64_t, bool, float*,
                                                 float*, hipStream_t);
template hipError_t launch_coupling_sweep<double>(const RowRec*, const Entry<double>*, int64_t, int64_t, bool,
                                                  double*, double*, hipStream_t);
template hipError_t launch_coupling_sweep<Cx<float>>(const RowRec*, const Entry<Cx<float>>*, int64_t, int64_t, bool,
                                                     Cx<float>*, Cx<float>*, hipStream_t);
template hipError_t launch_coupling_sweep<Cx<double>>(const RowRec*, const Entry<Cx<double>>*, int64_t, int64_t,
                                                      bool, Cx<double>*, Cx<double>*, hipStream_t);

}  // namespace mcinv
