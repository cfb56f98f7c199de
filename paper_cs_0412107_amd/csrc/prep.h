// Host-side preparation of one matrix for the sweep kernels (shared by the
// single-matrix context and the batched form).
//
//   - validation: sorted, duplicate-free columns; every row has a nonzero
//     diagonal (the sweep divides by c_ii; Sec. 2.2 needs D regular);
//   - the transpose of C (eq 5 walks column i of C);
//   - one merged off-diagonal pattern per row, the union of row i and column
//     i, holding u = c_ij/c_ii (eq 4) and v = conj(c_ji)/conj(c_ii) (eq 5);
//   - greedy first-fit colouring of that pattern in natural row order and the
//     position order (colour, row) -- a symmetric permutation of C;
//   - noise scales with a conj(b) = 1/c_ii (fp64).
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "device_common.h"

namespace mcinv {

using cd = std::complex<double>;

struct MergedEntry {
    int64_t col;   // position of the neighbour
    cd u, v;
};

struct Prepared {
    int64_t n = 0, nnz = 0;
    int32_t ncolors = 0;
    std::vector<int64_t> perm, pos, color_ptr;
    std::vector<int32_t> color;
    std::vector<RowRec> rows;       // per position; begin relative to this matrix
    std::vector<MergedEntry> ent;   // per position, columns ascending
    std::vector<cd> a, b;           // per position
    std::vector<cd> diag;           // c_ii per position
};

// Run f(begin, end) over [0, n) split into contiguous ranges on up to 16
// host threads (serially for small n).  Every stage below writes disjoint
// outputs per index, so the result does not depend on the split.
template <typename F>
inline void parallel_for(int64_t n, F&& f)
{
    constexpr int64_t kGrain = 1 << 14;
    int64_t T = std::min<int64_t>(16, std::max<unsigned>(1u, std::thread::hardware_concurrency()));
    T = std::min<int64_t>(T, n / kGrain);
    if (T <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)T);
    for (int64_t t = 0; t < T; ++t) th.emplace_back([&f, n, t, T]() { f(n * t / T, n * (t + 1) / T); });
    for (std::thread& x : th) x.join();
}

// Validation of a CSR matrix: sorted, duplicate-free, in-range columns and a
// nonzero diagonal in every row, which is returned in diag.  Rows are checked
// in parallel ranges; the reported failure is the lowest row's pattern error,
// else the lowest row without a diagonal.  Returns an empty string on success, else the
// reason; *singular is set when the failure is a missing or zero diagonal.
inline std::string validate_csr(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                                const double* vd, bool complex_values, std::vector<cd>& diag, bool* singular)
{
    *singular = false;
    if (n < 1 || n > INT32_MAX || nnz < n || !row_ptr || !col_idx || !vd) return "bad sizes or null arrays";
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return "row_ptr[0] must be 0 and row_ptr[n] nnz";
    for (int64_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return "row_ptr is decreasing";
    diag.assign(n, cd(0.0, 0.0));
    // per row: 0 fine, 1 column out of range, 2 columns not increasing, 3 no nonzero diagonal
    std::vector<int8_t> bad(n, 0);
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            bool found = false;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1] && !bad[i]; ++e) {
                if (col_idx[e] < 0 || col_idx[e] >= n)
                    bad[i] = 1;
                else if (e > row_ptr[i] && col_idx[e] <= col_idx[e - 1])
                    bad[i] = 2;
                else if (col_idx[e] == i) {
                    diag[i] = complex_values ? cd(vd[2 * e], vd[2 * e + 1]) : cd(vd[e], 0.0);
                    found = true;
                }
            }
            if (!bad[i] && (!found || diag[i] == cd(0.0, 0.0))) bad[i] = 3;
        }
    });
    for (int64_t i = 0; i < n; ++i) {   // pattern errors first, then a missing diagonal
        if (bad[i] == 1) return "column index out of range";
        if (bad[i] == 2) return "columns must be strictly increasing within a row";
    }
    for (int64_t i = 0; i < n; ++i)
        if (bad[i] == 3) {
            *singular = true;
            return "row " + std::to_string(i) + " has no nonzero diagonal entry";
        }
    return "";
}

// Transpose of the pattern: column i lists (row j, position of c_ji in the
// CSR arrays), rows ascending -- a counting sort over row ranges: range t
// counts its entries per column, the per-column counts become per-range
// offsets, then every range writes its own slots (ranges ascend, so rows come
// out ascending).
inline void transpose_csr(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                          std::vector<int64_t>& tptr, std::vector<int32_t>& trow, std::vector<int64_t>& tsrc)
{
    tptr.assign(n + 1, 0);
    trow.resize(nnz);
    tsrc.resize(nnz);
    // ranges: one per 16K rows, at most 16, and at most 2^25 / n (count memory)
    const int64_t T = std::max<int64_t>(1, std::min<int64_t>({16, n >> 14, ((int64_t)1 << 25) / n}));
    std::vector<int32_t> cnt((size_t)(T * n), 0);
    auto range_of = [&](int64_t t, int64_t* i0, int64_t* i1) {
        *i0 = n * t / T;
        *i1 = n * (t + 1) / T;
    };
    auto per_range = [&](auto&& body) {
        std::vector<std::thread> th;
        for (int64_t t = 1; t < T; ++t) th.emplace_back([&body, t]() { body(t); });
        body(0);
        for (std::thread& x : th) x.join();
    };
    per_range([&](int64_t t) {
        int64_t i0, i1;
        range_of(t, &i0, &i1);
        int32_t* c = cnt.data() + t * n;
        for (int64_t e = row_ptr[i0]; e < row_ptr[i1]; ++e) c[col_idx[e]]++;
    });
    parallel_for(n, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            int32_t run = 0;
            for (int64_t t = 0; t < T; ++t) {
                const int32_t k = cnt[t * n + c];
                cnt[t * n + c] = run;
                run += k;
            }
            tptr[c + 1] = run;
        }
    });
    for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    per_range([&](int64_t t) {
        int64_t i0, i1;
        range_of(t, &i0, &i1);
        int32_t* c = cnt.data() + t * n;
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                const int64_t slot = tptr[col_idx[e]] + c[col_idx[e]]++;
                trow[slot] = (int32_t)i;
                tsrc[slot] = e;
            }
    });
}

// Returns an empty string on success, else the reason; *singular is set when
// the failure is a missing or zero diagonal.
inline std::string prepare_matrix(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                                  const double* vd, bool complex_values, Prepared& h, bool* singular)
{
    std::vector<cd> diag;
    const std::string why = validate_csr(n, nnz, row_ptr, col_idx, vd, complex_values, diag, singular);
    if (!why.empty()) return why;
    auto val = [&](int64_t e) { return complex_values ? cd(vd[2 * e], vd[2 * e + 1]) : cd(vd[e], 0.0); };

    std::vector<int64_t> tptr;
    std::vector<int32_t> trow;
    std::vector<int64_t> tsrc;
    transpose_csr(n, nnz, row_ptr, col_idx, tptr, trow, tsrc);

    // Merged off-diagonal pattern per original row: the union of row i and
    // column i (both ascending).  merge_row visits it in column order;
    // emit(j, u, v) receives each neighbour j != i with its two coefficients.
    auto merge_row = [&](int64_t i, auto&& emit) {
        const cd inv = 1.0 / diag[i];
        const double inv_re = 1.0 / diag[i].real();   // real C: the same products without complex arithmetic
        int64_t e = row_ptr[i], t = tptr[i];
        const int64_t e_end = row_ptr[i + 1], t_end = tptr[i + 1];
        while (e < e_end || t < t_end) {
            const int64_t je = e < e_end ? col_idx[e] : INT64_MAX;
            const int64_t jt = t < t_end ? trow[t] : INT64_MAX;
            const int64_t j = std::min(je, jt);
            const bool has_e = je == j, has_t = jt == j;
            if (j != i) {
                cd u(0.0, 0.0), v(0.0, 0.0);
                if (complex_values) {
                    if (has_e) u = inv * val(e);
                    if (has_t) v = std::conj(inv) * std::conj(val(tsrc[t]));
                } else {
                    if (has_e) u = cd(inv_re * vd[e], 0.0);
                    if (has_t) v = cd(inv_re * vd[tsrc[t]], 0.0);
                }
                emit(j, u, v);
            }
            e += has_e ? 1 : 0;
            t += has_t ? 1 : 0;
        }
    };
    std::vector<int32_t> mcount(n);
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            int32_t k = 0;
            // count only: the coefficients are not needed yet
            int64_t e = row_ptr[i], t = tptr[i];
            const int64_t e_end = row_ptr[i + 1], t_end = tptr[i + 1];
            while (e < e_end || t < t_end) {
                const int64_t je = e < e_end ? col_idx[e] : INT64_MAX;
                const int64_t jt = t < t_end ? trow[t] : INT64_MAX;
                const int64_t j = std::min(je, jt);
                k += j != i ? 1 : 0;
                e += je == j ? 1 : 0;
                t += jt == j ? 1 : 0;
            }
            mcount[i] = k;
        }
    });

    // Greedy first-fit colouring in natural order (neighbours read from row i
    // and column i directly; a neighbour listed twice only marks twice).
    std::vector<int32_t> color(n, 0);
    std::vector<int64_t> mark(n + 1, -1);
    int32_t ncolors = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col_idx[e] < i) mark[color[col_idx[e]]] = i;
        for (int64_t t = tptr[i]; t < tptr[i + 1]; ++t)
            if (trow[t] < i) mark[color[trow[t]]] = i;
        int32_t k = 0;
        while (mark[k] == i) ++k;
        color[i] = k;
        ncolors = std::max(ncolors, k + 1);
    }
    std::vector<int64_t> color_ptr(ncolors + 1, 0);
    for (int64_t i = 0; i < n; ++i) color_ptr[color[i] + 1]++;
    for (int32_t k = 0; k < ncolors; ++k) color_ptr[k + 1] += color_ptr[k];
    std::vector<int64_t> perm(n), pos(n);
    {
        std::vector<int64_t> fill(color_ptr.begin(), color_ptr.end() - 1);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t q = fill[color[i]]++;
            perm[q] = i;
            pos[i] = q;
        }
    }

    h.n = n;
    h.nnz = nnz;
    h.ncolors = ncolors;
    h.rows.resize(n);
    h.a.resize(n);
    h.b.resize(n);
    h.diag.resize(n);
    std::vector<int64_t> begin(n + 1, 0);
    for (int64_t q = 0; q < n; ++q) begin[q + 1] = begin[q] + mcount[perm[q]];
    h.ent.resize((size_t)begin[n]);
    // rows in original order (sequential reads of C and its transpose), each
    // written to its position's slot
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            const int64_t q = pos[i];
            h.rows[q].begin = begin[q];
            h.rows[q].count = mcount[i];
            h.rows[q].orig = (uint32_t)i;
            MergedEntry* out = h.ent.data() + begin[q];
            int32_t k = 0;
            merge_row(i, [&](int64_t j, const cd& u, const cd& v) { out[k++] = MergedEntry{pos[j], u, v}; });
            for (int32_t a = 1; a < k; ++a)   // rows are short: insertion sort by position
                for (int32_t b = a; b > 0 && out[b - 1].col > out[b].col; --b) std::swap(out[b - 1], out[b]);
            const cd d = diag[i];
            h.diag[q] = d;
            if (!complex_values) {
                const double sc = 1.0 / std::sqrt(std::fabs(d.real()));
                h.a[q] = cd(sc, 0.0);
                h.b[q] = cd(d.real() > 0 ? sc : -sc, 0.0);
            } else {
                h.a[q] = 1.0 / std::sqrt(d);
                h.b[q] = std::conj(h.a[q]);
            }
        }
    });
    h.perm = std::move(perm);
    h.pos = std::move(pos);
    h.color = std::move(color);
    h.color_ptr = std::move(color_ptr);
    return "";
}

// Message returned by mcinv_last_error(NULL) (entry points without a context).
void set_context_free_error(const std::string& msg);

template <typename V> V cast_val(cd x);
template <> inline float cast_val<float>(cd x) { return (float)x.real(); }
template <> inline double cast_val<double>(cd x) { return x.real(); }
template <> inline Cx<float> cast_val<Cx<float>>(cd x) { return Cx<float>{(float)x.real(), (float)x.imag()}; }
template <> inline Cx<double> cast_val<Cx<double>>(cd x) { return Cx<double>{x.real(), x.imag()}; }

}  // namespace mcinv
