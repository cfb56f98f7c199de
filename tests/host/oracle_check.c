/* The oracle's C part (Philox noise, greedy colouring, sweeps with moment
 * accumulation) built with the address and undefined-behaviour sanitizers by
 * tests/test_host_sanitizers_cpu.py: a random non-symmetric matrix through
 * colouring, burn-in and sampling with every moment kind, a complex matrix,
 * and a matrix without a diagonal entry (refused). */
#include "../../oracle/mcinv_oracle.c"

#include <stdio.h>

static uint32_t lcg(uint32_t* s) { *s = *s * 1664525u + 1013904223u; return *s >> 8; }

static int run(int64_t n, int is_complex, int drop_diag_row)
{
    uint32_t st = 12345u + (uint32_t)n;
    int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n * 5));
    double* val = (double*)malloc(sizeof(double) * (size_t)(n * 5 * 2));
    int64_t nnz = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t cs[5];
        int k = 0;
        cs[k++] = (int32_t)i;
        for (int t = 0; t < 4; ++t) cs[k++] = (int32_t)(lcg(&st) % (uint32_t)n);
        /* sort and drop duplicates */
        for (int a = 1; a < k; ++a)
            for (int b = a; b > 0 && cs[b - 1] > cs[b]; --b) { int32_t x = cs[b]; cs[b] = cs[b - 1]; cs[b - 1] = x; }
        for (int a = 0; a < k; ++a) {
            if (a > 0 && cs[a] == cs[a - 1]) continue;
            if (drop_diag_row >= 0 && i == drop_diag_row && cs[a] == i) continue;
            col[nnz] = cs[a];
            double v = cs[a] == i ? 6.0 : ((double)(lcg(&st) % 1000) / 1000.0 - 0.5);
            if (is_complex) { val[2 * nnz] = v; val[2 * nnz + 1] = cs[a] == i ? 0.5 : 0.1 * v; }
            else val[nnz] = v;
            ++nnz;
        }
        rp[i + 1] = nnz;
    }
    int32_t* color = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t ncolors = 0;
    ora_greedy_color(n, rp, col, color, order, &ncolors);
    const int64_t P = 6, S = 5, nb = 2;
    int64_t pids[6] = {0, 1, 2, 3, 4, 5};
    double* z = (double*)calloc((size_t)(n * P * 2), sizeof(double));
    double* w = (double*)calloc((size_t)(n * P * 2), sizeof(double));
    int64_t bI[3] = {0, n / 2, n - 1}, bJ[2] = {1 % n, n - 1}, ei[2] = {0, n - 1}, ej[2] = {n - 1, 0};
    ora_moments m;
    memset(&m, 0, sizeof(m));
    m.groups = 2; m.pairs_total = P; m.batch_len = 3; m.n_batches = nb; m.want_diag = 1;
    m.diag = (double*)calloc((size_t)(nb * 2 * n * 2), sizeof(double));
    m.nI = 3; m.nJ = 2; m.bI = bI; m.bJ = bJ;
    m.block = (double*)calloc((size_t)(nb * 2 * 3 * 2 * 2), sizeof(double));
    m.n_entries = 2; m.ei = ei; m.ej = ej;
    m.entries = (double*)calloc((size_t)(nb * 2 * 2 * 2), sizeof(double));
    m.max_samples = S; m.trace_series = (double*)calloc((size_t)(S * 2), sizeof(double));
    m.cluster_count = (double*)calloc((size_t)(nb * 2), sizeof(double));
    int s1 = ora_sweeps(n, rp, col, val, is_complex, order, 7u, 0u, 0, P, pids, z, w, 0, 3, NULL);
    int s2 = s1 == ORA_OK ? ora_sweeps(n, rp, col, val, is_complex, order, 7u, 0u, 1, P, pids, z, w, 3, S, &m) : s1;
    free(rp); free(col); free(val); free(color); free(order); free(z); free(w);
    free(m.diag); free(m.block); free(m.entries); free(m.trace_series); free(m.cluster_count);
    return s2;
}

int main(void)
{
    int fails = 0;
    if (run(1, 0, -1) != ORA_OK) ++fails;
    if (run(300, 0, -1) != ORA_OK) ++fails;
    if (run(120, 1, -1) != ORA_OK) ++fails;
    if (run(80, 0, 17) != ORA_ESINGULAR) ++fails;
    printf("oracle_check: %d failures\n", fails);
    return fails == 0 ? 0 : 1;
}
