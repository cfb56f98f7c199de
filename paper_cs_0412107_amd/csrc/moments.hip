// Moment accumulation and finalisation kernels (eq 1/C, eq tr, Sec. 2.3).
//
//  - k_block_fp64: dense requested block, sum over each chain group of
//    z[I_r][p] conj(w[J_t][p]) in fp64, 32 x 32 output tile per workgroup with
//    LDS-staged z and w tiles.
//  - k_entries: an arbitrary list of (i, j) entries.
//  - k_merge_slots: doubles the time-batch length of the error clusters.
//  - k_reduce_sum: deterministic two-stage sum (per-sweep trace value).
//  - k_finalize_*: cluster ratio estimator -> estimate and standard error.
//  - k_geyer: Geyer's initial positive sequence on the trace series.
#include "device_common.h"
#include "moments.h"
#include "sweep.h"

namespace mcinv {

template <typename V> struct Wide;
template <> struct Wide<float> { using type = double; };
template <> struct Wide<double> { using type = double; };
template <> struct Wide<Cx<float>> { using type = Cx<double>; };
template <> struct Wide<Cx<double>> { using type = Cx<double>; };

__device__ inline double widen(float x) { return x; }
__device__ inline double widen(double x) { return x; }
__device__ inline Cx<double> widen(Cx<float> x) { return Cx<double>{x.re, x.im}; }
__device__ inline Cx<double> widen(Cx<double> x) { return x; }

// acc + x conj(y)
__device__ inline double conj_fma(double x, double y, double acc) { return __builtin_fma(x, y, acc); }
__device__ inline Cx<double> conj_fma(Cx<double> x, Cx<double> y, Cx<double> acc)
{
    acc.re = __builtin_fma(x.re, y.re, acc.re);
    acc.re = __builtin_fma(x.im, y.im, acc.re);
    acc.im = __builtin_fma(x.im, y.re, acc.im);
    acc.im = __builtin_fma(-x.re, y.im, acc.im);
    return acc;
}

__device__ inline void add_to(double* p, double v) { p[0] += v; }
__device__ inline void add_to(double* p, Cx<double> v)
{
    p[0] += v.re;
    p[1] += v.im;
}

// ------------------------------------------------------------------ block --
constexpr int kBT = 32;  // output tile edge
constexpr int kBK = 32;  // pairs per LDS stage

template <typename V>
__global__ __launch_bounds__(256) void k_block_fp64(const BlockArgs<V> a)
{
    using W = typename Wide<V>::type;
    constexpr int comps = IsCx<V>::value ? 2 : 1;
    __shared__ W zs[kBT][kBK + 1];
    __shared__ W ws[kBT][kBK + 1];

    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int64_t r0 = (int64_t)blockIdx.y * kBT;
    const int64_t t0 = (int64_t)blockIdx.x * kBT;
    const int64_t g = blockIdx.z;
    const int64_t pbeg = g * a.gs, pend = pbeg + a.gs;

    W acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = vzero<W>();

    const int lr = tid >> 3;         // row of the tile this thread loads
    const int lk = (tid & 7) * 4;    // first pair of the four it loads
    const int64_t zrow = (r0 + lr < a.nI) ? a.I[r0 + lr] : -1;
    const int64_t wrow = (t0 + lr < a.nJ) ? a.J[t0 + lr] : -1;

    for (int64_t kb = pbeg; kb < pend; kb += kBK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t p = kb + lk + e;
            const bool ok = p < pend;
            zs[lr][lk + e] = (ok && zrow >= 0) ? widen(a.z[zrow * a.ld + p]) : vzero<W>();
            ws[lr][lk + e] = (ok && wrow >= 0) ? widen(a.w[wrow * a.ld + p]) : vzero<W>();
        }
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < kBK; ++k) {
            const W z0 = zs[ty][k], z1 = zs[ty + 16][k];
            const W w0 = ws[tx][k], w1 = ws[tx + 16][k];
            acc[0][0] = conj_fma(z0, w0, acc[0][0]);
            acc[0][1] = conj_fma(z0, w1, acc[0][1]);
            acc[1][0] = conj_fma(z1, w0, acc[1][0]);
            acc[1][1] = conj_fma(z1, w1, acc[1][1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t r = r0 + ty + 16 * i;
        if (r >= a.nI) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t t = t0 + tx + 16 * j;
            if (t >= a.nJ) continue;
            add_to(a.acc + comps * ((g * a.nI + r) * a.nJ + t), acc[i][j]);
        }
    }
}

template <typename V>
hipError_t launch_block_fp64(const BlockArgs<V>& a, hipStream_t stream)
{
    if (a.nI <= 0 || a.nJ <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.nJ + kBT - 1) / kBT), (unsigned)((a.nI + kBT - 1) / kBT), (unsigned)a.G);
    k_block_fp64<V><<<grid, dim3(256), 0, stream>>>(a);
    return hipGetLastError();
}
template hipError_t launch_block_fp64<float>(const BlockArgs<float>&, hipStream_t);
template hipError_t launch_block_fp64<double>(const BlockArgs<double>&, hipStream_t);
template hipError_t launch_block_fp64<Cx<float>>(const BlockArgs<Cx<float>>&, hipStream_t);
template hipError_t launch_block_fp64<Cx<double>>(const BlockArgs<Cx<double>>&, hipStream_t);

// ---------------------------------------------------------------- entries --
template <typename V>
__global__ __launch_bounds__(256) void k_entries(const V* z, const V* w, int64_t ld, const int64_t* ei,
                                                 const int64_t* ej, int64_t ne, int64_t gs, int64_t G,
                                                 double* acc)
{
    using W = typename Wide<V>::type;
    constexpr int comps = IsCx<V>::value ? 2 : 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * G) return;
    const int64_t e = t % ne, g = t / ne;
    const V* zr = z + ei[e] * ld;
    const V* wr = w + ej[e] * ld;
    W s = vzero<W>();
    for (int64_t p = g * gs; p < (g + 1) * gs; ++p) s = conj_fma(widen(zr[p]), widen(wr[p]), s);
    add_to(acc + comps * (g * ne + e), s);
}

template <typename V>
hipError_t launch_entries(const V* z, const V* w, int64_t ld, const int64_t* ei, const int64_t* ej, int64_t ne,
                          int64_t gs, int64_t G, double* acc, hipStream_t stream)
{
    if (ne <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((ne * G + 255) / 256);
    k_entries<V><<<dim3(blocks), dim3(256), 0, stream>>>(z, w, ld, ei, ej, ne, gs, G, acc);
    return hipGetLastError();
}
template hipError_t launch_entries<float>(const float*, const float*, int64_t, const int64_t*, const int64_t*,
                                          int64_t, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_entries<double>(const double*, const double*, int64_t, const int64_t*,
                                           const int64_t*, int64_t, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_entries<Cx<float>>(const Cx<float>*, const Cx<float>*, int64_t, const int64_t*,
                                              const int64_t*, int64_t, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_entries<Cx<double>>(const Cx<double>*, const Cx<double>*, int64_t, const int64_t*,
                                               const int64_t*, int64_t, int64_t, int64_t, double*, hipStream_t);

// ---------------------------------------------------------------- Q trace --
// Per-sample value of w^dagger Q z summed over the chain pairs (eq tr with a
// general sparse Q): a wave takes kQRowsPerWave consecutive rows q of Q
// (position order) and 256 pairs, forms each (Q z)_q in fp64 and multiplies by
// conj(w_q); one fp64 partial (x2 complex) per workgroup at
// part[(tile * gridDim.x + row block) * comps].
template <typename V>
__global__ __launch_bounds__(256) void k_qtrace(const QTraceArgs<V> a)
{
    using W = typename Wide<V>::type;
    constexpr int comps = IsCx<V>::value ? 2 : 1;
    __shared__ double lds[4][2];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t p0 = (int64_t)blockIdx.y * kPairsPerWave + lane * kPairsPerLane;
    W t = vzero<W>();
    for (int r = 0; r < kQRowsPerWave; ++r) {
        const int64_t q = ((int64_t)blockIdx.x * 4 + wid) * kQRowsPerWave + r;
        if (q >= a.n || p0 >= a.ld) break;
        W acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = vzero<W>();
        for (int64_t e = a.qrp[q]; e < a.qrp[q + 1]; ++e) {
            const W qv = widen(a.qval[e]);
            const V* zr = a.z + a.qcol[e] * a.ld + p0;
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = mul_add(qv, widen(zr[j]), acc[j]);
        }
        const V* wr = a.w + q * a.ld + p0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (p0 + j < a.P) t = conj_fma(acc[j], widen(wr[j]), t);
    }
    double re, im = 0.0;
    if constexpr (comps == 2) {
        re = t.re;
        im = t.im;
    } else {
        re = t;
    }
    for (int off = 1; off < 64; off <<= 1) {
        re += __shfl_xor(re, off);
        if constexpr (comps == 2) im += __shfl_xor(im, off);
    }
    if (lane == 0) {
        lds[wid][0] = re;
        lds[wid][1] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t slot = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        a.part[slot * comps] = ((lds[0][0] + lds[1][0]) + lds[2][0]) + lds[3][0];
        if constexpr (comps == 2) a.part[slot * 2 + 1] = ((lds[0][1] + lds[1][1]) + lds[2][1]) + lds[3][1];
    }
}

template <typename V>
hipError_t launch_qtrace(const QTraceArgs<V>& a, hipStream_t stream)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t rows_per_block = 4 * kQRowsPerWave;
    const dim3 grid((unsigned)((a.n + rows_per_block - 1) / rows_per_block),
                    (unsigned)((a.ld + kPairsPerWave - 1) / kPairsPerWave));
    k_qtrace<V><<<grid, dim3(256), 0, stream>>>(a);
    return hipGetLastError();
}
template hipError_t launch_qtrace<float>(const QTraceArgs<float>&, hipStream_t);
template hipError_t launch_qtrace<double>(const QTraceArgs<double>&, hipStream_t);
template hipError_t launch_qtrace<Cx<float>>(const QTraceArgs<Cx<float>>&, hipStream_t);
template hipError_t launch_qtrace<Cx<double>>(const QTraceArgs<Cx<double>>&, hipStream_t);

// ------------------------------------------------------------ slot merge --
// One thread per element walks the slots upwards: slot m is written only
// after slots 2m and 2m+1 (both >= m) were read, so the update is in place.
__global__ __launch_bounds__(256) void k_merge_slots(double* acc, int64_t slot_elems, int64_t half)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= slot_elems) return;
    for (int64_t m = 0; m < half; ++m)
        acc[m * slot_elems + e] = acc[(2 * m) * slot_elems + e] + acc[(2 * m + 1) * slot_elems + e];
    for (int64_t m = half; m < 2 * half; ++m) acc[m * slot_elems + e] = 0.0;
}

// max_q |x[q * ld]| over n rows (lane 0 of each row) as the bits of a
// non-negative double (their integer order is the value order); non-finite
// values count as +inf.
__device__ inline double modulus(float x) { return fabs((double)x); }
__device__ inline double modulus(double x) { return fabs(x); }
template <typename R> __device__ inline double modulus(Cx<R> x)
{
    return sqrt((double)x.re * (double)x.re + (double)x.im * (double)x.im);
}

template <typename V>
__global__ __launch_bounds__(256) void k_max_abs(const V* x, int64_t n, int64_t ld, unsigned long long* out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (q < n) {
        v = modulus(x[q * ld]);
        if (!(v < __builtin_inf())) v = __builtin_inf();
    }
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}

template <typename V>
hipError_t launch_max_abs(const V* x, int64_t n, int64_t ld, unsigned long long* out, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    k_max_abs<V><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream>>>(x, n, ld, out);
    return hipGetLastError();
}
template hipError_t launch_max_abs<float>(const float*, int64_t, int64_t, unsigned long long*, hipStream_t);
template hipError_t launch_max_abs<double>(const double*, int64_t, int64_t, unsigned long long*, hipStream_t);
template hipError_t launch_max_abs<Cx<float>>(const Cx<float>*, int64_t, int64_t, unsigned long long*, hipStream_t);
template hipError_t launch_max_abs<Cx<double>>(const Cx<double>*, int64_t, int64_t, unsigned long long*,
                                               hipStream_t);

hipError_t launch_merge_slots(double* acc, int64_t slot_elems, int64_t half, hipStream_t stream)
{
    if (slot_elems <= 0 || half <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((slot_elems + 255) / 256);
    k_merge_slots<<<dim3(blocks), dim3(256), 0, stream>>>(acc, slot_elems, half);
    return hipGetLastError();
}

// ------------------------------------------------------------ reductions --
template <int NT>
__device__ inline double block_sum(double v, double* lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

constexpr int kRedBlocks = 128;

// Stage 1: block b sums a fixed contiguous chunk; the last block to finish
// (atomic ticket) sums the kRedBlocks partials in order.  Deterministic.
__global__ __launch_bounds__(256) void k_reduce_sum(const double* x, int64_t count, int comps,
                                                     double* partial, uint32_t* counter, double* out)
{
    __shared__ double lds[256];
    __shared__ bool last;
    const int64_t chunk = (count + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < count ? beg + chunk : count;
    for (int c = 0; c < comps; ++c) {
        double s = 0.0;
        for (int64_t i = beg + threadIdx.x; i < end; i += 256) s += x[i * comps + c];
        s = block_sum<256>(s, lds);
        if (threadIdx.x == 0) partial[blockIdx.x * comps + c] = s;
    }
    __threadfence();
    if (threadIdx.x == 0) {
        const uint32_t ticket = atomicAdd(counter, 1u);
        last = ticket == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int c = 0; c < comps; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += 256)
            s += __hip_atomic_load(&partial[b * comps + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s = block_sum<256>(s, lds);
        if (threadIdx.x == 0) out[c] = s;
    }
    if (threadIdx.x == 0) *counter = 0u;
}

hipError_t launch_reduce_sum(const double* x, int64_t count, int comps, double* partial, uint32_t* counter,
                             double* out, hipStream_t stream)
{
    k_reduce_sum<<<dim3(kRedBlocks), dim3(256), 0, stream>>>(x, count, comps, partial, counter, out);
    return hipGetLastError();
}

// ------------------------------------------------------------- finalize --
// Ratio estimator over clusters c = (slot b, group g) with n_c = slot_len[b] gs
// terms and sum S_c:  est = sum S_c / sum n_c,
// Var = nc/(nc-1) sum_c (S_c - n_c est)^2 / (sum n_c)^2  (per real component).

// atomicMax of v >= 0 (double bits: non-negative doubles order like their
// bit patterns) into base[idx] for the lanes with has set.  Called by all 64
// lanes of a wave; when every such lane targets the same slot, the wave
// reduces first and issues one atomic (rows of one matrix share a slot, so
// per-lane atomics would serialise on it).
__device__ inline void wave_atomic_max(unsigned long long* base, int64_t idx, bool has, double v)
{
    const int64_t idx0 = __shfl(idx, __builtin_ctzll(__ballot(has) | (1ull << 63)));
    if (__all(!has || idx == idx0)) {
        double m = has ? v : -1.0;
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
        if ((threadIdx.x & 63) == 0 && m >= 0.0) atomicMax(base + idx0, (unsigned long long)__double_as_longlong(m));
    } else if (has) {
        atomicMax(base + idx, (unsigned long long)__double_as_longlong(v));
    }
}

__device__ inline double rel_error(double se, double er, double ei)
{
    double rel = se / sqrt(er * er + ei * ei);
    if (!(rel >= 0.0) || !(rel < __builtin_inf())) rel = __builtin_inf();
    return rel;
}

// Diagonal: one thread per position; groups gather their columns.  Returns
// whether the position counts for max_rel, with its se/|est| in *rel.
__device__ inline bool finalize_diag_row(const FinalizeArgs& f, int64_t q, double* rel)
{
    const int64_t ncl = f.nslots * f.G;
    const int64_t cols_per_group = f.G > 1 ? f.gs / f.pairs_per_col : f.A;
    // Sums are formed on the fly per cluster (two passes).
    double wsum = 0.0, er = 0.0, ei = 0.0;
    int64_t nc = 0;
    for (int64_t c = 0; c < ncl; ++c) {
        const int64_t b = c / f.G, g = c % f.G;
        const double wt = f.slot_len[b] * (double)f.gs;
        if (wt <= 0.0) continue;
        const double* slot = f.acc + b * f.slot_stride;
        double sr = 0.0, si = 0.0;
        for (int64_t k = g * cols_per_group; k < (g + 1) * cols_per_group && k < f.A; ++k) {
            const double* v = slot + (((k / f.cpt) * f.M + q) * f.cpt + k % f.cpt) * f.comps;
            sr += v[0];
            if (f.comps == 2) si += v[1];
        }
        wsum += wt;
        er += sr;
        ei += si;
        ++nc;
    }
    const int64_t out = f.out_index[q];
    const bool stop_row = f.max_rel != nullptr && (f.stop_mask == nullptr || f.stop_mask[out] != 0);
    if (wsum <= 0.0) {
        f.est[out * f.comps] = __builtin_nan("");
        if (f.comps == 2) f.est[out * 2 + 1] = __builtin_nan("");
        f.se[out] = __builtin_nan("");
        *rel = __builtin_inf();
        return stop_row;
    }
    er /= wsum;
    ei /= wsum;
    double vr = 0.0, vi = 0.0;
    for (int64_t c = 0; c < ncl; ++c) {
        const int64_t b = c / f.G, g = c % f.G;
        const double wt = f.slot_len[b] * (double)f.gs;
        if (wt <= 0.0) continue;
        const double* slot = f.acc + b * f.slot_stride;
        double sr = 0.0, si = 0.0;
        for (int64_t k = g * cols_per_group; k < (g + 1) * cols_per_group && k < f.A; ++k) {
            const double* v = slot + (((k / f.cpt) * f.M + q) * f.cpt + k % f.cpt) * f.comps;
            sr += v[0];
            if (f.comps == 2) si += v[1];
        }
        const double dr = sr - wt * er;
        vr += dr * dr;
        if (f.comps == 2) {
            const double di = si - wt * ei;
            vi += di * di;
        }
    }
    double se = __builtin_nan("");
    if (nc >= 2) se = sqrt((vr + vi) * ((double)nc / (double)(nc - 1))) / wsum;
    f.est[out * f.comps] = er;
    if (f.comps == 2) f.est[out * 2 + 1] = ei;
    f.se[out] = se;
    *rel = rel_error(se, er, ei);
    return stop_row;
}

__global__ __launch_bounds__(64) void k_finalize_diag(const FinalizeArgs f)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rel = 0.0;
    const bool has = q < f.M && finalize_diag_row(f, q, &rel);
    if (f.max_rel) wave_atomic_max(f.max_rel, 0, has, rel);
}

// Flat accumulators: value m of group g in slot b at
// acc[b * slot_stride + (g * gstride + m * mstride) * comps]; one thread per value.
__device__ inline void finalize_flat_value(const FinalizeArgs& f, int64_t m0, double* rel)
{
    const int64_t gstride = f.gstride > 0 ? f.gstride : f.M;
    const int64_t mstride = f.mstride > 0 ? f.mstride : 1;
    const int64_t ncl = f.nslots * f.G;
    const int64_t m = f.out_index ? f.out_index[m0] : m0;  // output index
    const double* slot_len = f.slot_len;
    double wsum = 0.0, er = 0.0, ei = 0.0;
    int64_t nc = 0;
    for (int64_t c = 0; c < ncl; ++c) {
        const double wt = slot_len[c / f.G] * (double)f.gs;
        if (wt <= 0.0) continue;
        const double* v = f.acc + (c / f.G) * f.slot_stride + ((c % f.G) * gstride + m0 * mstride) * f.comps;
        wsum += wt;
        er += v[0];
        if (f.comps == 2) ei += v[1];
        ++nc;
    }
    if (wsum <= 0.0) {
        f.est[m * f.comps] = __builtin_nan("");
        if (f.comps == 2) f.est[m * 2 + 1] = __builtin_nan("");
        f.se[m] = __builtin_nan("");
        *rel = __builtin_inf();
        return;
    }
    er /= wsum;
    ei /= wsum;
    double vr = 0.0, vi = 0.0;
    for (int64_t c = 0; c < ncl; ++c) {
        const double wt = slot_len[c / f.G] * (double)f.gs;
        if (wt <= 0.0) continue;
        const double* v = f.acc + (c / f.G) * f.slot_stride + ((c % f.G) * gstride + m0 * mstride) * f.comps;
        const double dr = v[0] - wt * er;
        vr += dr * dr;
        if (f.comps == 2) {
            const double di = v[1] - wt * ei;
            vi += di * di;
        }
    }
    double se = __builtin_nan("");
    if (nc >= 2) se = sqrt((vr + vi) * ((double)nc / (double)(nc - 1))) / wsum;
    f.est[m * f.comps] = er;
    if (f.comps == 2) f.est[m * 2 + 1] = ei;
    f.se[m] = se;
    *rel = rel_error(se, er, ei);
}

__global__ __launch_bounds__(64) void k_finalize_flat(const FinalizeArgs f)
{
    const int64_t m0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool has = m0 < f.M;
    double rel = 0.0;
    if (has) finalize_flat_value(f, m0, &rel);
    if (f.max_rel) wave_atomic_max(f.max_rel, 0, has, rel);
}

// Flat accumulators laid out [nslots][M][G] with G a power of two <= 64
// (gstride 1, mstride G): a wave takes 64/G values, lane = (value, group), so
// every load is coalesced and a value's sums are butterfly reductions over its
// G lanes.  Same estimator as k_finalize_flat (sums in another order).
__global__ __launch_bounds__(256) void k_finalize_groups(const FinalizeArgs f)
{
    const int G = (int)f.G;
    const int lg = __builtin_ctz((unsigned)G);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = t >> lg;
    const int g = (int)(t & (G - 1));
    const bool ok = v < f.M;
    const int64_t grp = ok && f.val_group ? f.val_group[v] : 0;
    const double* slot_len = f.slot_len + grp * f.slot_len_stride;
    double wsum = 0.0, er = 0.0, ei = 0.0, nc = 0.0;
    double x0r = 0.0, x0i = 0.0, w0 = 0.0;   // the only slot's cluster when there is one (no second read)
    if (ok)
        for (int64_t b = 0; b < f.nslots; ++b) {
            const double wt = slot_len[b] * (double)f.gs;
            if (wt <= 0.0) continue;
            const double* x = f.acc + b * f.slot_stride + (v * G + g) * f.comps;
            x0r = x[0];
            if (f.comps == 2) x0i = x[1];
            w0 = wt;
            wsum += wt;
            er += x0r;
            ei += x0i;
            nc += 1.0;
        }
    for (int off = 1; off < G; off <<= 1) {
        wsum += __shfl_xor(wsum, off);
        er += __shfl_xor(er, off);
        ei += __shfl_xor(ei, off);
        nc += __shfl_xor(nc, off);
    }
    double vr = 0.0, vi = 0.0;
    if (ok && wsum > 0.0) {
        const double mr = er / wsum, mi = ei / wsum;
        if (f.nslots == 1) {
            const double dr = x0r - w0 * mr, di = x0i - w0 * mi;
            vr = dr * dr;
            vi = f.comps == 2 ? di * di : 0.0;
        } else {
            for (int64_t b = 0; b < f.nslots; ++b) {
                const double wt = slot_len[b] * (double)f.gs;
                if (wt <= 0.0) continue;
                const double* x = f.acc + b * f.slot_stride + (v * G + g) * f.comps;
                const double dr = x[0] - wt * mr;
                vr += dr * dr;
                if (f.comps == 2) {
                    const double di = x[1] - wt * mi;
                    vi += di * di;
                }
            }
        }
    }
    for (int off = 1; off < G; off <<= 1) {
        vr += __shfl_xor(vr, off);
        vi += __shfl_xor(vi, off);
    }
    const bool has = ok && g == 0;
    double rel = 0.0;
    if (has) {
        // est / se may be null (a stop check needs only rel): no scattered writes then
        const int64_t m = f.out_index ? f.out_index[v] : v;
        if (wsum <= 0.0) {
            if (f.est) {
                f.est[m * f.comps] = __builtin_nan("");
                if (f.comps == 2) f.est[m * 2 + 1] = __builtin_nan("");
                f.se[m] = __builtin_nan("");
            }
            rel = __builtin_inf();
        } else {
            const double mr = er / wsum, mi = ei / wsum;
            double se = __builtin_nan("");
            if (nc >= 2.0) se = sqrt((vr + vi) * (nc / (nc - 1.0))) / wsum;
            if (f.est) {
                f.est[m * f.comps] = mr;
                if (f.comps == 2) f.est[m * 2 + 1] = mi;
                f.se[m] = se;
            }
            rel = rel_error(se, mr, mi);
        }
    }
    if (has && f.rel_out) f.rel_out[v] = rel;
}

// out[s] = max of x[begin[s] .. begin[s+1]) (values >= 0, NaN taken as +inf;
// 0 for an empty segment); one workgroup per segment, no atomics.
__global__ __launch_bounds__(256) void k_segment_max(const double* x, const int64_t* begin, double* out)
{
    __shared__ double lds[256];
    const int64_t seg = blockIdx.x;
    double m = 0.0;
    for (int64_t i = begin[seg] + threadIdx.x; i < begin[seg + 1]; i += 256) {
        const double v = x[i];
        m = fmax(m, v <= __builtin_inf() ? v : __builtin_inf());
    }
    lds[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[seg] = lds[0];
}

hipError_t launch_segment_max(const double* x, const int64_t* begin, int64_t nseg, double* out, hipStream_t stream)
{
    if (nseg <= 0) return hipSuccess;
    k_segment_max<<<dim3((unsigned)nseg), dim3(256), 0, stream>>>(x, begin, out);
    return hipGetLastError();
}

hipError_t launch_finalize_groups(const FinalizeArgs& f, hipStream_t stream)
{
    if (f.M <= 0) return hipSuccess;
    if (f.G < 1 || f.G > 64 || (f.G & (f.G - 1)) != 0) return hipErrorInvalidValue;
    const int64_t threads = f.M * f.G;
    k_finalize_groups<<<dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream>>>(f);
    return hipGetLastError();
}

hipError_t launch_finalize_diag(const FinalizeArgs& f, hipStream_t stream)
{
    if (f.M <= 0) return hipSuccess;
    k_finalize_diag<<<dim3((unsigned)((f.M + 63) / 64)), dim3(64), 0, stream>>>(f);
    return hipGetLastError();
}

hipError_t launch_finalize_flat(const FinalizeArgs& f, hipStream_t stream)
{
    if (f.M <= 0) return hipSuccess;
    k_finalize_flat<<<dim3((unsigned)((f.M + 63) / 64)), dim3(64), 0, stream>>>(f);
    return hipGetLastError();
}

// ----------------------------------------------------------------- Geyer --
// gamma_t = (1/S) sum_{k < S-t} (x_k - mean)(x_{k+t} - mean); pairs
// Gamma_m = gamma_2m + gamma_2m+1 are summed while positive;
// sigma^2 = -gamma_0 + 2 sum Gamma_m; SE = sqrt(sigma^2 / S).
__global__ __launch_bounds__(1024) void k_geyer(const double* x, int64_t S, int comps, double scale,
                                                double* out)
{
    __shared__ double lds[1024];
    double g0_tot = 0.0, sig_tot = 0.0, mean[2] = {0.0, 0.0}, g0c[2] = {0.0, 0.0};
    for (int c = 0; c < comps; ++c) {
        double s = 0.0;
        for (int64_t k = threadIdx.x; k < S; k += 1024) s += x[k * comps + c] * scale;
        const double mu = block_sum<1024>(s, lds) / (double)S;
        mean[c] = mu;
        auto gamma = [&](int64_t t) {
            double acc = 0.0;
            for (int64_t k = threadIdx.x; k + t < S; k += 1024)
                acc += (x[k * comps + c] * scale - mu) * (x[(k + t) * comps + c] * scale - mu);
            return block_sum<1024>(acc, lds) / (double)S;
        };
        const double g0 = gamma(0);
        double sig2 = -g0;
        for (int64_t m = 0; 2 * m + 1 < S; ++m) {
            const double pair_sum = gamma(2 * m) + gamma(2 * m + 1);
            if (!(pair_sum > 0.0)) break;
            sig2 += 2.0 * pair_sum;
        }
        if (!(sig2 > 0.0)) sig2 = g0;
        g0c[c] = g0;
        g0_tot += g0;
        sig_tot += sig2;
    }
    if (threadIdx.x == 0) {
        out[0] = mean[0];
        out[1] = mean[1];
        out[2] = g0_tot;
        out[3] = sig_tot;
        out[4] = sig_tot > 0.0 ? (double)S * g0_tot / sig_tot : __builtin_nan("");
        out[5] = S >= 2 ? sqrt(sig_tot / (double)S) : __builtin_nan("");
        out[6] = g0c[0];   // gamma_0 of the real part
        out[7] = g0c[1];   // and of the imaginary part (0 for a real series)
    }
}

hipError_t launch_geyer(const double* series, int64_t S, int comps, double scale, double* out,
                        hipStream_t stream)
{
    k_geyer<<<dim3(1), dim3(1024), 0, stream>>>(series, S, comps, scale, out);
    return hipGetLastError();
}

}  // namespace mcinv
