// Host-side check of the matrix preparation (validation, transpose, merged
// pattern, greedy colouring, position order), built with the address and
// undefined-behaviour sanitizers by tests/test_host_sanitizers_cpu.py.
// Random sparse matrices (empty off-diagonal rows, a long hub row, one-sided
// entries) must prepare without sanitizer reports, and the result must be a
// valid multicolouring: a permutation, colours contiguous, no merged entry
// joining two rows of one colour, each row's merged list ascending and equal
// to the union of its row and column.  Invalid inputs must be refused.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "prep.h"

namespace mcinv {
void set_context_free_error(const std::string&) {}
}

using namespace mcinv;

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                     \
        }                                                                \
    } while (0)

struct Csr {
    int64_t n;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<double> val;
};

static Csr random_matrix(int64_t n, int per_row, bool hub, uint32_t seed)
{
    std::mt19937 rng(seed);
    std::vector<std::set<int32_t>> rows(n);
    for (int64_t i = 0; i < n; ++i) {
        rows[i].insert((int32_t)i);
        if (i % 7 == 3) continue;   // rows with no off-diagonal entry of their own
        for (int k = 0; k < per_row; ++k) rows[i].insert((int32_t)(rng() % n));
    }
    if (hub)
        for (int64_t j = 0; j < n; ++j) rows[0].insert((int32_t)j);
    Csr m{n, {0}, {}, {}};
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t j : rows[i]) {
            m.col.push_back(j);
            m.val.push_back(j == i ? 3.0 + per_row : 0.5 - (double)(rng() % 1000) / 1000.0);
        }
        m.rp.push_back((int64_t)m.col.size());
    }
    return m;
}

static void check_prepared(const Csr& m, const Prepared& h)
{
    const int64_t n = m.n;
    CHECK(h.n == n && (int64_t)h.perm.size() == n && (int64_t)h.pos.size() == n);
    std::vector<char> seen(n, 0);
    for (int64_t q = 0; q < n; ++q) {
        CHECK(h.perm[q] >= 0 && h.perm[q] < n && !seen[h.perm[q]]);
        seen[h.perm[q]] = 1;
        CHECK(h.pos[h.perm[q]] == q);
    }
    for (int32_t k = 0; k < h.ncolors; ++k)
        for (int64_t q = h.color_ptr[k]; q < h.color_ptr[k + 1]; ++q) CHECK(h.color[h.perm[q]] == k);
    // merged lists: union of row i and column i (without i), ascending positions, no same-colour pair
    std::vector<std::set<int64_t>> want(n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = m.rp[i]; e < m.rp[i + 1]; ++e)
            if (m.col[e] != i) {
                want[i].insert(m.col[e]);
                want[m.col[e]].insert(i);
            }
    for (int64_t q = 0; q < n; ++q) {
        const RowRec& r = h.rows[q];
        const int64_t i = h.perm[q];
        CHECK((int64_t)r.orig == i && r.count == (int32_t)want[i].size());
        std::set<int64_t> got;
        for (int32_t t = 0; t < r.count; ++t) {
            const int64_t pcol = h.ent[r.begin + t].col;
            if (t > 0) CHECK(h.ent[r.begin + t - 1].col < pcol);
            CHECK(h.color[h.perm[pcol]] != h.color[i]);
            got.insert(h.perm[pcol]);
        }
        CHECK(got == want[i]);
    }
}

int main()
{
    const int64_t sizes[] = {1, 2, 50, 20000, 70000};
    uint32_t seed = 7;
    for (int64_t n : sizes)
        for (bool hub : {false, true}) {
            const Csr m = random_matrix(n, 3, hub, seed++);
            Prepared h;
            bool singular = false;
            const std::string why = prepare_matrix(n, (int64_t)m.col.size(), m.rp.data(), m.col.data(),
                                                   m.val.data(), false, h, &singular);
            CHECK(why.empty());
            if (why.empty()) check_prepared(m, h);
        }
    // invalid inputs are refused, not read out of bounds
    Csr bad = random_matrix(300, 3, false, 99);
    bad.col[bad.rp[5]] = 400;   // column out of range
    Prepared h;
    bool singular = false;
    CHECK(!prepare_matrix(bad.n, (int64_t)bad.col.size(), bad.rp.data(), bad.col.data(), bad.val.data(), false, h,
                          &singular).empty());
    Csr dec = random_matrix(300, 3, false, 98);
    std::swap(dec.rp[10], dec.rp[11]);   // decreasing row pointers
    CHECK(!prepare_matrix(dec.n, (int64_t)dec.col.size(), dec.rp.data(), dec.col.data(), dec.val.data(), false, h,
                          &singular).empty());
    std::printf("prep_check: %d failures\n", fails);
    return fails == 0 ? 0 : 1;
}
