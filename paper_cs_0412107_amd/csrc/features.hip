// Local features of each row for the learned surrogate of diag(C^-1).
//
// With C = D (I + M), M = D^-1 R (R the off-diagonal part), the Neumann series
// gives c_ii (C^-1)_ii = 1 + (M^2)_ii - (M^3)_ii + ...; the features are local
// terms of that series and neighbourhood statistics (list in include/mcinv.h,
// mcinv_features).  Pass 1 computes the per-row terms; pass 2 the statistics
// over each row's merged neighbours (row i or column i of C) from pass 1's
// output.  fp64 arithmetic (pass 1: eight lanes per row; pass 2: one thread
// per row), fp32 output.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mcinv.h"
#include "boundary.h"
#include "prep.h"
#include "surrogate_internal.h"

namespace mcinv {

constexpr int kNF = 32;

struct FEnt {
    int32_t col;   // position of the neighbour
    int32_t pad;
    double cij;    // c_ij (row entry), 0 if not stored
    double cji;    // c_ji (column entry), 0 if not stored
};

// c_ki for neighbour k of row i: binary search of k in i's sorted merged list.
__device__ inline double lookup_cji(const FEnt* e, int32_t cnt, int32_t k)
{
    int lo = 0, hi = cnt - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int32_t c = e[mid].col;
        if (c == k) return e[mid].cji;
        if (c < k)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return 0.0;
}

// The merged neighbour lists are built on the device.  The transpose of C is
// a counting sort by column: column counts, their prefix sums (column
// pointers), a scatter of every entry into its column's segment (slots taken
// with atomics, so in no fixed order), then each entry's rank among its
// segment's rows puts the segment in ascending row order -- the same result
// whatever order the scatter took.

// Validation of the CSR arrays (thread per row) and the diagonal c_ii.
// flag[0]: lowest row with a pattern error (-1: row_ptr does not start at 0 or
// end at nnz); flag[1]: lowest row without a nonzero diagonal; both start at
// INT64_MAX.  Row ranges outside [0, nnz] are flagged and not read.
__global__ __launch_bounds__(256) void k_ft_validate(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
                                                     const double* val, double* d, unsigned long long* flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicMin(flag, 0ull);
    if (i >= n) return;
    const int64_t b = rp[i], e = rp[i + 1];
    bool bad = b < 0 || e < b || e > nnz;
    bool found = false;
    double di = 0.0;
    for (int64_t k = b; k < e && !bad; ++k) {
        const int32_t c = col[k];
        if (c < 0 || c >= n || (k > b && c <= col[k - 1]))
            bad = true;
        else if (c == i) {
            di = val[k];
            found = true;
        }
    }
    if (bad) {
        atomicMin(flag, (unsigned long long)(i + 1));
        return;
    }
    d[i] = di;
    if (!found || di == 0.0) atomicMin(flag + 1, (unsigned long long)i);
}

template <typename T>
__global__ __launch_bounds__(256) void k_ft_fill(int64_t count, T* p, T v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = v;
}

// entry count of every column (thread per row)
__global__ __launch_bounds__(256) void k_ft_colcount(int64_t n, const int64_t* rp, const int32_t* col,
                                                     int32_t* ccount)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) atomicAdd(ccount + col[e], 1);
}

// every entry c_ij into column j's segment (cursor: zeroed counts)
__global__ __launch_bounds__(256) void k_ft_scatter(int64_t n, const int64_t* rp, const int32_t* col,
                                                    const double* val, const int64_t* tp, int32_t* cursor,
                                                    int32_t* trow_u, int32_t* tcol_u, double* tval_u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t j = col[e];
        const int64_t at = tp[j] + atomicAdd(cursor + j, 1);
        trow_u[at] = (int32_t)i;
        tcol_u[at] = j;
        tval_u[at] = val[e];
    }
}

// thread per transposed entry: its rank among the rows of its column (rows
// are distinct within a column) is its place in ascending order
__global__ __launch_bounds__(256) void k_ft_rank(int64_t nnz, const int64_t* tp, const int32_t* trow_u,
                                                 const int32_t* tcol_u, const double* tval_u, int32_t* trow,
                                                 double* tval)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnz) return;
    const int32_t j = tcol_u[t], r = trow_u[t];
    const int64_t b = tp[j], e = tp[j + 1];
    int64_t rank = 0;
    for (int64_t u = b; u < e; ++u) rank += trow_u[u] < r ? 1 : 0;
    trow[b + rank] = r;
    tval[b + rank] = tval_u[t];
}

// out[k] = in[0] + ... + in[k-1] for k = 0..n (one workgroup: a chunk per
// thread, the chunk sums scanned in LDS); used on the per-tile sums below
template <typename T>
__global__ __launch_bounds__(1024) void k_ft_scan(int64_t n, const T* in, int64_t* out)
{
    __shared__ int64_t part[1024];
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = (int64_t)threadIdx.x * per, e = b + per < n ? b + per : n;
    int64_t s = 0;
    for (int64_t k = b; k < e; ++k) s += (int64_t)in[k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int64_t k = b; k < e; ++k) {
        out[k] = run;
        run += (int64_t)in[k];
    }
    if (threadIdx.x == 1023) out[n] = part[1023];
}

// Exclusive scan of int32 counts over tiles of 1024: the tiles' sums, their
// scan (k_ft_scan), then each tile's own scan plus its offset.
__global__ __launch_bounds__(1024) void k_ft_tile_sums(int64_t n, const int32_t* in, int64_t* sums)
{
    __shared__ int64_t ws[16];
    const int64_t k = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    int64_t v = k < n ? (int64_t)in[k] : 0;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < 16; ++w) t += ws[w];
        sums[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_ft_tile_scan(int64_t n, const int32_t* in, const int64_t* offs,
                                                       int64_t* out)
{
    __shared__ int64_t ws[16];
    const int64_t k = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t x = k < n ? (int64_t)in[k] : 0;
    int64_t v = x;   // inclusive scan within the wave
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(v, off);
        if (lane >= off) v += y;
    }
    if (lane == 63) ws[w] = v;
    __syncthreads();
    int64_t before = offs[blockIdx.x];
    for (int q = 0; q < w; ++q) before += ws[q];
    if (k < n) out[k] = before + v - x;
    if (k == n - 1) out[n] = before + v;
}

// out[0..n] = exclusive prefix sums of in[0..n); tsum / toff hold
// ceil(n / 1024) and ceil(n / 1024) + 1 values
inline hipError_t scan_counts(int64_t n, const int32_t* in, int64_t* out, int64_t* tsum, int64_t* toff,
                              hipStream_t st)
{
    const int64_t nt = (n + 1023) / 1024;
    k_ft_tile_sums<<<(unsigned)nt, 1024, 0, st>>>(n, in, tsum);
    k_ft_scan<int64_t><<<1, 1024, 0, st>>>(nt, tsum, toff);
    k_ft_tile_scan<<<(unsigned)nt, 1024, 0, st>>>(n, in, toff, out);
    return hipGetLastError();
}

// Row i's merged list: the union of row i (col, val) and column i (rows
// trow[tp[i] .. tp[i+1]), ascending, with values tval), ascending, without i
// itself.
// Counting pass (out == nullptr) writes cnt[i]; the writing pass fills
// out + beg[i].
__global__ __launch_bounds__(256) void k_ft_merge(int64_t n, const int64_t* rp, const int32_t* col,
                                                  const double* val, const int64_t* tp, const int32_t* trow,
                                                  const double* tval, const int64_t* beg, FEnt* out, int32_t* cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t e = rp[i], t = tp[i];
    const int64_t e_end = rp[i + 1], t_end = tp[i + 1];
    FEnt* o = out ? out + beg[i] : nullptr;
    int32_t k = 0;
    while (e < e_end || t < t_end) {
        const int64_t je = e < e_end ? (int64_t)col[e] : INT64_MAX;
        const int64_t jt = t < t_end ? (int64_t)trow[t] : INT64_MAX;
        const int64_t j = je < jt ? je : jt;
        const bool has_e = je == j, has_t = jt == j;
        if (j != i) {
            if (o) o[k] = FEnt{(int32_t)j, 0, has_e ? val[e] : 0.0, has_t ? tval[t] : 0.0};
            ++k;
        }
        e += has_e ? 1 : 0;
        t += has_t ? 1 : 0;
    }
    if (!o) cnt[i] = k;
}

// Pass 1: kRowLanes lanes per row, each taking every kRowLanes-th merged
// neighbour; the partial sums meet in an xor-shuffle tree within the lane
// group (fixed order, so the result is deterministic).
constexpr int kRowLanes = 8;

__global__ __launch_bounds__(256) void k_features_pass1(int64_t n, const int64_t* beg, const int32_t* cnt,
                                                        const FEnt* ent, const double* d, double* F)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = gid / kRowLanes;
    const int lane = (int)(gid % kRowLanes);
    const bool valid = i < n;   // a lane group lies in one row, so groups are wholly valid or not
    const FEnt* e = valid ? ent + beg[i] : ent;
    const int32_t c = valid ? cnt[i] : 0;
    const double di = valid ? d[i] : 1.0;
    double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // rs cs nr nc m2 m3 a2 sq srow scol (unused)
    for (int32_t t = lane; t < c; t += kRowLanes) {
        const int32_t j = e[t].col;
        const double cij = e[t].cij, cji = e[t].cji, dj = d[j];
        v[0] += fabs(cij);
        v[1] += fabs(cji);
        v[2] += cij != 0.0 ? 1.0 : 0.0;
        v[3] += cji != 0.0 ? 1.0 : 0.0;
        const double mij = cij / di, mji = cji / dj;
        v[4] += mij * mji;
        v[6] += fabs(mij) * fabs(mji);
        v[7] += mij * mij;
        v[8] += cij;
        v[9] += cji;
        if (cij != 0.0) {
            // sum_k m_jk m_ki over the stored entries of row j
            const FEnt* ej = ent + beg[j];
            const int32_t cj = cnt[j];
            double inner = 0.0;
            for (int32_t u = 0; u < cj; ++u) {
                const int32_t k = ej[u].col;
                if (k == (int32_t)i || ej[u].cij == 0.0) continue;
                const double cki = lookup_cji(e, c, k);
                inner += (ej[u].cij / dj) * (cki / d[k]);
            }
            v[5] += mij * inner;
        }
    }
#pragma unroll
    for (int q = 0; q < 10; ++q)
        for (int off = 1; off < kRowLanes; off <<= 1) v[q] += __shfl_xor(v[q], off);
    if (!valid || lane != 0) return;
    const double adi = fabs(di);
    const double rs = v[0], cs = v[1], nr = v[2], nc = v[3], m2 = v[4], m3 = v[5], a2 = v[6], sq = v[7],
                 srow = v[8], scol = v[9];
    double* f = F + i * kNF;
    f[0] = log(adi);
    f[1] = rs / adi;
    f[2] = cs / adi;
    f[3] = nr / 8.0;
    f[4] = nc / 8.0;
    f[5] = m2;
    f[6] = m3;
    f[7] = a2;
    f[8] = sq;
    f[9] = srow / di;
    f[10] = scol / di;
    f[24] = c / 8.0;
    f[25] = 1.0 + m2;
    f[26] = 1.0 + m2 - m3;
    f[27] = f[1] * f[1];
    f[28] = m2 * m2;
    f[29] = m2 * f[1];
    f[31] = 1.0;
}

__device__ inline void stats(double v, double& s1, double& s2, double& mx, double& mn)
{
    s1 += v;
    s2 += v * v;
    mx = fmax(mx, v);
    mn = fmin(mn, v);
}

__global__ __launch_bounds__(256) void k_features_pass2(int64_t n, const int64_t* beg, const int32_t* cnt,
                                                        const FEnt* ent, double* F, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const FEnt* e = ent + beg[i];
    const int32_t c = cnt[i];
    double* f = F + i * kNF;
    double r1 = 0, r2 = 0, rmx = -INFINITY, rmn = INFINITY;   // neighbours' row ratio
    double l1 = 0, l2 = 0, lmx = -INFINITY, lmn = INFINITY;   // neighbours' log|c_jj|
    double q1 = 0, q2 = 0, qmx = -INFINITY, qmn = INFINITY;   // neighbours' (M^2)_jj
    double c1 = 0, c2 = 0, cmx = -INFINITY, cmn = INFINITY;   // neighbours' column ratio
    double t1 = 0;                                            // neighbours' (M^3)_jj
    for (int32_t t = 0; t < c; ++t) {
        const double* g = F + (int64_t)e[t].col * kNF;
        stats(g[1], r1, r2, rmx, rmn);
        stats(g[0], l1, l2, lmx, lmn);
        stats(g[5], q1, q2, qmx, qmn);
        stats(g[2], c1, c2, cmx, cmn);
        t1 += g[6];
    }
    double o[kNF];
    for (int k = 0; k < kNF; ++k) o[k] = f[k];
    if (c > 0) {
        const double rm = r1 / c, lm = l1 / c;
        // population standard deviations from the squared deviations (a second
        // pass: no cancellation when the neighbours' values are all equal)
        double rv = 0.0, lv = 0.0;
        for (int32_t t = 0; t < c; ++t) {
            const double* g = F + (int64_t)e[t].col * kNF;
            rv += (g[1] - rm) * (g[1] - rm);
            lv += (g[0] - lm) * (g[0] - lm);
        }
        o[11] = rm;
        o[12] = rmx;
        o[13] = rmn;
        o[14] = sqrt(rv / c);
        o[15] = lm - f[0];
        o[16] = lmx - f[0];
        o[17] = lmn - f[0];
        o[18] = sqrt(lv / c);
        o[19] = q1 / c;
        o[20] = qmx;
        o[21] = c1 / c;
        o[22] = cmx;
        o[23] = t1 / c;
    } else {
        for (int k = 11; k <= 23; ++k) o[k] = 0.0;
    }
    o[30] = r2 / 8.0;
    float* dst = out + i * kNF;
    for (int k = 0; k < kNF; ++k) dst[k] = (float)o[k];
}

__global__ __launch_bounds__(256) void k_ft_pick(int64_t n, const float* F, int32_t a, int32_t b, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[2 * i] = F[i * kNF + a];
    out[2 * i + 1] = F[i * kNF + b];
}

// Device buffers of one features computation, all carved (256-byte aligned)
// from one region: its size for a matrix of n rows and nnz entries, and the
// carving.  The merged lists take the bound 2 nnz (every entry in both its
// row's and its column's list).
struct FeatBuffers {
    int32_t* ccount;                 // n: column counts, then scatter cursors
    int64_t* tp;                     // n + 1: column pointers
    int32_t *trow_u, *tcol_u;        // nnz: scattered entries
    double* tval_u;                  // nnz
    int32_t* trow;                   // nnz: rows ascending within each column
    double* tval;                    // nnz
    int32_t* cnt;                    // n: merged list lengths
    int64_t* beg;                    // n + 1: merged list offsets
    double* d;                       // n: c_ii
    double* F;                       // n x 32: pass-1 terms
    int64_t *tsum, *toff;            // scan tiles
    FEnt* ent;                       // 2 nnz: merged lists
    unsigned long long* flag;        // 2: validation
};

template <class F>
void feat_parts(int64_t n, int64_t nnz, F&& part)
{
    const size_t N = (size_t)n, Z = (size_t)nnz, T = (size_t)((n + 1023) / 1024);
    part(0, sizeof(int32_t) * N);
    part(1, sizeof(int64_t) * (N + 1));
    part(2, sizeof(int32_t) * Z);
    part(3, sizeof(int32_t) * Z);
    part(4, sizeof(double) * Z);
    part(5, sizeof(int32_t) * Z);
    part(6, sizeof(double) * Z);
    part(7, sizeof(int32_t) * N);
    part(8, sizeof(int64_t) * (N + 1));
    part(9, sizeof(double) * N);
    part(10, sizeof(double) * N * kNF);
    part(11, sizeof(int64_t) * std::max<size_t>(T, 1));
    part(12, sizeof(int64_t) * (T + 1));
    part(13, sizeof(FEnt) * std::max<size_t>(2 * Z, 1));
    part(14, sizeof(unsigned long long) * 2);
}

inline size_t pad256(size_t b) { return (b + 255) / 256 * 256; }

size_t feat_bytes(int64_t n, int64_t nnz)
{
    size_t total = 0;
    feat_parts(n, nnz, [&](int, size_t b) { total += pad256(b); });
    return total;
}

FeatBuffers feat_carve(char* base, int64_t n, int64_t nnz)
{
    void* at[15];
    size_t off = 0;
    feat_parts(n, nnz, [&](int k, size_t b) {
        at[k] = base + off;
        off += pad256(b);
    });
    FeatBuffers f;
    f.ccount = (int32_t*)at[0];
    f.tp = (int64_t*)at[1];
    f.trow_u = (int32_t*)at[2];
    f.tcol_u = (int32_t*)at[3];
    f.tval_u = (double*)at[4];
    f.trow = (int32_t*)at[5];
    f.tval = (double*)at[6];
    f.cnt = (int32_t*)at[7];
    f.beg = (int64_t*)at[8];
    f.d = (double*)at[9];
    f.F = (double*)at[10];
    f.tsum = (int64_t*)at[11];
    f.toff = (int64_t*)at[12];
    f.ent = (FEnt*)at[13];
    f.flag = (unsigned long long*)at[14];
    return f;
}

inline unsigned grid_for(int64_t count) { return (unsigned)((std::max<int64_t>(count, 1) + 255) / 256); }

// Validation on the device (the diagonal into fb.d); the flags are read back
// with a synchronisation: flag[0] / flag[1] as k_ft_validate writes them.
hipError_t features_validate(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col, const double* val,
                             const FeatBuffers& fb, unsigned long long flags[2], hipStream_t st)
{
    k_ft_fill<unsigned long long><<<1, 256, 0, st>>>(2, fb.flag, ~0ull);
    k_ft_validate<<<grid_for(n), 256, 0, st>>>(n, nnz, rp, col, val, fb.d, fb.flag);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(flags, fb.flag, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// Status and message of the validation flags.
mcinv_status validation_status(const unsigned long long flags[2], const char** why)
{
    if (flags[0] != ~0ull) {
        *why = flags[0] == 0 ? "row_ptr[0] must be 0 and row_ptr[n] nnz"
                             : "a row has a bad entry range, a column out of range or columns not strictly "
                               "increasing";
        return MCINV_EINVAL;
    }
    if (flags[1] != ~0ull) {
        *why = "a row has no nonzero diagonal entry";
        return MCINV_ESINGULAR;
    }
    return MCINV_OK;
}

// The features of a validated matrix (device CSR arrays; fb.d holds c_ii)
// into out [n][32] float, all launches on st.
hipError_t features_kernels(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col, const double* val,
                            const FeatBuffers& fb, float* out, hipStream_t st)
{
    const unsigned rows = grid_for(n);
    k_ft_fill<int32_t><<<rows, 256, 0, st>>>(n, fb.ccount, 0);
    k_ft_colcount<<<rows, 256, 0, st>>>(n, rp, col, fb.ccount);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = scan_counts(n, fb.ccount, fb.tp, fb.tsum, fb.toff, st);
    if (e != hipSuccess) return e;
    k_ft_fill<int32_t><<<rows, 256, 0, st>>>(n, fb.ccount, 0);
    k_ft_scatter<<<rows, 256, 0, st>>>(n, rp, col, val, fb.tp, fb.ccount, fb.trow_u, fb.tcol_u, fb.tval_u);
    k_ft_rank<<<grid_for(nnz), 256, 0, st>>>(nnz, fb.tp, fb.trow_u, fb.tcol_u, fb.tval_u, fb.trow, fb.tval);
    k_ft_merge<<<rows, 256, 0, st>>>(n, rp, col, val, fb.tp, fb.trow, fb.tval, nullptr, nullptr, fb.cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_counts(n, fb.cnt, fb.beg, fb.tsum, fb.toff, st)) != hipSuccess) return e;
    k_ft_merge<<<rows, 256, 0, st>>>(n, rp, col, val, fb.tp, fb.trow, fb.tval, fb.beg, fb.ent, fb.cnt);
    k_ft_fill<double><<<grid_for(n * kNF), 256, 0, st>>>(n * kNF, fb.F, 0.0);
    k_features_pass1<<<grid_for(n * kRowLanes), 256, 0, st>>>(n, fb.beg, fb.cnt, fb.ent, fb.d, fb.F);
    k_features_pass2<<<rows, 256, 0, st>>>(n, fb.beg, fb.cnt, fb.ent, fb.F, out);
    return hipGetLastError();
}

mcinv_status features_on_device(int32_t device, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                const int32_t* col_idx, const double* values, float** d_features, std::string* err,
                                std::vector<double>* diag_out)
{
    *d_features = nullptr;
    std::vector<cd> diag;
    bool singular = false;
    const std::string why = validate_csr(n, nnz, row_ptr, col_idx, values, false, diag, &singular);
    if (!why.empty()) {
        *err = why;
        return singular ? MCINV_ESINGULAR : MCINV_EINVAL;
    }
    if (diag_out) {
        diag_out->resize(n);
        for (int64_t i = 0; i < n; ++i) (*diag_out)[i] = diag[i].real();
    }
    if (hipSetDevice(device) != hipSuccess) {
        *err = "no such device";
        return MCINV_EDEVICE;
    }
    // device buffers, released on every exit (the features buffer is handed over on success)
    struct Owned {
        std::vector<void*> p;
        ~Owned()
        {
            for (void* x : p) (void)hipFree(x);
        }
    } owned;
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t bytes) {
        *p = nullptr;
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 1));
        if (e == hipSuccess) owned.p.push_back(*p);
    };
    // the CSR copy and every scratch buffer are parts of one allocation (few
    // allocations per call: small matrices are called many times)
    const size_t csr_bytes = pad256(sizeof(int64_t) * (n + 1)) + pad256(sizeof(int32_t) * nnz) +
                             pad256(sizeof(double) * nnz);
    char* slab = nullptr;
    float* d_out = nullptr;
    alloc((void**)&slab, csr_bytes + feat_bytes(n, nnz));
    alloc((void**)&d_out, sizeof(float) * (size_t)n * kNF);
    if (e == hipSuccess) {
        int64_t* d_rp = (int64_t*)slab;
        int32_t* d_col = (int32_t*)(slab + pad256(sizeof(int64_t) * (n + 1)));
        double* d_val = (double*)((char*)d_col + pad256(sizeof(int32_t) * nnz));
        const FeatBuffers fb = feat_carve(slab + csr_bytes, n, nnz);
        e = hipMemcpy(d_rp, row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_col, col_idx, sizeof(int32_t) * nnz, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_val, values, sizeof(double) * nnz, hipMemcpyHostToDevice);
        unsigned long long flags[2] = {0, 0};
        if (e == hipSuccess) e = features_validate(n, nnz, d_rp, d_col, d_val, fb, flags, nullptr);
        if (e == hipSuccess) {
            const char* w = nullptr;
            const mcinv_status vs = validation_status(flags, &w);
            if (vs != MCINV_OK) {   // the host check above passed, so the two disagree
                *err = std::string("device validation: ") + w;
                return MCINV_EINTERNAL;
            }
        }
        if (e == hipSuccess) e = features_kernels(n, nnz, d_rp, d_col, d_val, fb, d_out, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    }
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? MCINV_ENOMEM : MCINV_EDEVICE;
    }
    owned.p.erase(std::find(owned.p.begin(), owned.p.end(), (void*)d_out));
    *d_features = d_out;
    return MCINV_OK;
}

mcinv_status features_pick_two(const float* d_features, int64_t n, int32_t a, int32_t b, float* out,
                               std::string* err)
{
    float* d2 = nullptr;
    hipError_t e = hipMalloc((void**)&d2, sizeof(float) * 2 * (size_t)std::max<int64_t>(n, 1));
    if (e == hipSuccess && n > 0) {
        k_ft_pick<<<(unsigned)((n + 255) / 256), 256>>>(n, d_features, a, b, d2);
        e = hipGetLastError();
    }
    if (e == hipSuccess && n > 0) e = hipMemcpy(out, d2, sizeof(float) * 2 * n, hipMemcpyDeviceToHost);
    if (d2) (void)hipFree(d2);
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? MCINV_ENOMEM : MCINV_EDEVICE;
    }
    return MCINV_OK;
}

}  // namespace mcinv

using namespace mcinv;

extern "C" mcinv_status mcinv_features(int32_t device, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                       const int32_t* col_idx, const double* values, float* out)
try {
    if (!out) {
        set_context_free_error("mcinv_features: null output");
        return MCINV_EINVAL;
    }
    float* d_F = nullptr;
    std::string why;
    const mcinv_status st = features_on_device(device, n, nnz, row_ptr, col_idx, values, &d_F, &why);
    if (st != MCINV_OK) {
        set_context_free_error("mcinv_features: " + why);
        return st;
    }
    const hipError_t e = hipMemcpy(out, d_F, sizeof(float) * n * kNF, hipMemcpyDeviceToHost);
    (void)hipFree(d_F);
    if (e != hipSuccess) {
        set_context_free_error(std::string("mcinv_features: ") + hipGetErrorString(e));
        return MCINV_EDEVICE;
    }
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status, const std::string& m_) { set_context_free_error(m_); });
}

// ---------------------------------------------------------------------------
// Features that allocate nothing: the caller's device arrays in and out, the
// scratch buffers carved from a file-scope device array of fixed size.  Each
// GPU holds its own copy of the array; its address on a device comes from
// hipGetSymbolAddress on that device's first call (the array's name is only a
// host-side stand-in and never reaches a kernel).  Every call on a GPU reuses
// that GPU's array, so calls on one GPU must not overlap.
namespace {

constexpr int64_t kNoAllocMaxRows = 32768;
constexpr int64_t kNoAllocMaxNnz = 262144;
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
constexpr int kNoAllocMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

}  // namespace

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

// The scratch array's device address on the current device (looked up once per device).
hipError_t scratch_on(int32_t device, void** ptr)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" mcinv_status mcinv_features_noalloc(int32_t device, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                               const int32_t* col_idx, const double* values, float* out,
                                               void* stream)
try {
    if (!row_ptr || !col_idx || !values || !out) {
        set_context_free_error("mcinv_features_noalloc: null device array");
        return MCINV_EINVAL;
    }
    if (n < 1 || nnz < n || n > kNoAllocMaxRows || nnz > kNoAllocMaxNnz) {
        set_context_free_error("mcinv_features_noalloc: needs 1 <= n <= 32768 and n <= nnz <= 262144 (the "
                               "fixed scratch size); use mcinv_features for larger matrices");
        return MCINV_EINVAL;
    }
    static_assert(kNoAllocMaxRows <= INT32_MAX, "row indices are 32-bit");
    if (device < 0 || device >= kNoAllocMaxDevices || hipSetDevice(device) != hipSuccess) {
        set_context_free_error("mcinv_features_noalloc: no such device");
        return MCINV_EDEVICE;
    }
    void* base = nullptr;
    hipError_t e = scratch_on(device, &base);
    if (e == hipSuccess && feat_bytes(n, nnz) > kNoAllocScratchBytes) e = hipErrorInvalidValue;   // guarded above
    const hipStream_t st = (hipStream_t)stream;
    const FeatBuffers fb = feat_carve((char*)base, n, nnz);
    unsigned long long flags[2] = {0, 0};
    if (e == hipSuccess) e = features_validate(n, nnz, row_ptr, col_idx, values, fb, flags, st);
    if (e == hipSuccess) {
        const char* why = nullptr;
        const mcinv_status vs = validation_status(flags, &why);
        if (vs != MCINV_OK) {
            set_context_free_error(std::string("mcinv_features_noalloc: ") + why);
            return vs;
        }
        e = features_kernels(n, nnz, row_ptr, col_idx, values, fb, out, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_context_free_error(std::string("mcinv_features_noalloc: ") + hipGetErrorString(e));
        return MCINV_EDEVICE;
    }
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status, const std::string& m_) { set_context_free_error(m_); });
}
