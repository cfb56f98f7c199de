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

// Returns an empty string on success, else the reason; *singular is set when
// the failure is a missing or zero diagonal.
inline std::string prepare_matrix(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                                  const double* vd, bool complex_values, Prepared& h, bool* singular)
{
    *singular = false;
    if (n < 1 || n > INT32_MAX || nnz < n || !row_ptr || !col_idx || !vd) return "bad sizes or null arrays";
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return "row_ptr[0] must be 0 and row_ptr[n] nnz";
    for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return "row_ptr is decreasing";
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col_idx[e] < 0 || col_idx[e] >= n) return "column index out of range";
            if (e > row_ptr[i] && col_idx[e] <= col_idx[e - 1])
                return "columns must be strictly increasing within a row";
        }
    }
    auto val = [&](int64_t e) { return complex_values ? cd(vd[2 * e], vd[2 * e + 1]) : cd(vd[e], 0.0); };

    std::vector<cd> diag(n);
    for (int64_t i = 0; i < n; ++i) {
        bool found = false;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col_idx[e] == i) {
                diag[i] = val(e);
                found = true;
            }
        if (!found || diag[i] == cd(0.0, 0.0)) {
            *singular = true;
            return "row " + std::to_string(i) + " has no nonzero diagonal entry";
        }
    }

    // Transpose: column i lists (row j, position of c_ji), rows ascending.
    std::vector<int64_t> tptr(n + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) tptr[col_idx[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    std::vector<int64_t> trow(nnz), tsrc(nnz);
    {
        std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                const int64_t slot = fill[col_idx[e]]++;
                trow[slot] = i;
                tsrc[slot] = e;
            }
    }

    // Merged off-diagonal pattern per original row.
    std::vector<int64_t> mptr(n + 1, 0), mcol;
    std::vector<cd> mu, mv;
    mcol.reserve(2 * nnz);
    mu.reserve(2 * nnz);
    mv.reserve(2 * nnz);
    for (int64_t i = 0; i < n; ++i) {
        const cd inv = 1.0 / diag[i];
        int64_t e = row_ptr[i], t = tptr[i];
        const int64_t e_end = row_ptr[i + 1], t_end = tptr[i + 1];
        while (e < e_end || t < t_end) {
            const int64_t je = e < e_end ? col_idx[e] : INT64_MAX;
            const int64_t jt = t < t_end ? trow[t] : INT64_MAX;
            const int64_t j = std::min(je, jt);
            cd u(0.0, 0.0), v(0.0, 0.0);
            if (je == j) u = inv * val(e++);
            if (jt == j) v = std::conj(inv) * std::conj(val(tsrc[t++]));
            if (j == i) continue;
            mcol.push_back(j);
            mu.push_back(u);
            mv.push_back(v);
        }
        mptr[i + 1] = (int64_t)mcol.size();
    }

    // Greedy first-fit colouring in natural order.
    std::vector<int32_t> color(n, 0);
    std::vector<int64_t> mark(n + 1, -1);
    int32_t ncolors = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = mptr[i]; e < mptr[i + 1]; ++e)
            if (mcol[e] < i) mark[color[mcol[e]]] = i;
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
    h.rows.assign(n, RowRec{});
    h.a.assign(n, cd());
    h.b.assign(n, cd());
    h.diag.assign(n, cd());
    h.ent.clear();
    h.ent.reserve(mcol.size());
    for (int64_t q = 0; q < n; ++q) {
        const int64_t i = perm[q];
        h.rows[q].begin = (int64_t)h.ent.size();
        h.rows[q].count = (int32_t)(mptr[i + 1] - mptr[i]);
        h.rows[q].orig = (uint32_t)i;
        const size_t first = h.ent.size();
        for (int64_t e = mptr[i]; e < mptr[i + 1]; ++e) h.ent.push_back(MergedEntry{pos[mcol[e]], mu[e], mv[e]});
        std::sort(h.ent.begin() + first, h.ent.end(),
                  [](const MergedEntry& x, const MergedEntry& y) { return x.col < y.col; });
        const cd d = diag[i];
        h.diag[q] = d;
        if (!complex_values) {
            const double s = 1.0 / std::sqrt(std::fabs(d.real()));
            h.a[q] = cd(s, 0.0);
            h.b[q] = cd(d.real() > 0 ? s : -s, 0.0);
        } else {
            h.a[q] = 1.0 / std::sqrt(d);
            h.b[q] = std::conj(h.a[q]);
        }
    }
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
