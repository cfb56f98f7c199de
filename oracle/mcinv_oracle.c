/*
 * Correlated-chains Monte Carlo matrix inverter -- CPU ORACLE.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg load this file.  It is a plain, slow,
 * single-threaded double-precision (complex128) implementation written from
 * the paper (Garcia-Cortes & Cabrillo, "A Monte Carlo algorithm for efficient
 * large matrix inversion"), and it shares no code with the GPU library.
 *
 *   - Noisy coupled Gauss-Seidel sweep:   Sec. 2, eqs (4) and (5)
 *   - Noise properties:                   Sec. 2, eqs (5a), (5b)
 *   - Inverse / trace estimators:         Sec. 2, eqs (1/C) and (tr)
 *   - Initial values z = w = 0:           Sec. 2.4, Algorithm 1, step 1
 *
 * Readings taken where the paper is loose:
 *   - the noise is N(0,1) from Philox4x32-10 (Salmon et al., SC'11) turned into
 *     normals by the Box-Muller transform (Box & Muller, 1958), or Z2 noise
 *     (+1/-1, the noise preferred in the introduction);
 *   - the z and w noise scales a_i, b_i only need a_i * conj(b_i) = 1/c_ii
 *     (the step "sqrt(D) sqrt(D) = D" of the demonstration, Sec. 2.1):
 *     real c_ii: a = 1/sqrt|c_ii|, b = sign(c_ii) a;  complex: a = 1/sqrt(c_ii)
 *     (principal root), b = conj(a) -- equal to 1/sqrt(conj c_ii) off the cut;
 *   - the sweep visits rows in a caller-given order (a symmetric permutation
 *     P C P^T of the matrix, still eqs (4)-(5) on the permuted matrix);
 *   - entry (i,j) of the inverse is estimated by z_i conj(w_j) and the trace by
 *     sum_i z_i conj(w_i) (= w^dagger z, whose expectation is tr C^-1).
 *
 * The CPU tests pin this file to closed forms, exact special cases and dense
 * LU inverses (tests/test_oracle_*.py).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
 * multiply-xorshift bijection with a Weyl-sequence key schedule.            */
/* ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1): the top 23 bits plus one half, times 2^-23 (exact in
 * binary32 as well as binary64). */
double ora_uniform(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

enum { ORA_NOISE_NORMAL = 0, ORA_NOISE_RADEMACHER = 1, ORA_NOISE_NONE = 2 };

/* The four noise values of one Philox block.  Counter = (row, sweep, pair/4,
 * stream), key = (seed low word, seed high word). */
void ora_noise_block(uint64_t seed, uint32_t stream, uint32_t row, uint32_t sweep,
                     uint32_t quad, int kind, double out[4])
{
    uint32_t ctr[4] = {row, sweep, quad, stream};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    ora_philox4x32_10(ctr, key, x);
    if (kind == ORA_NOISE_NONE) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
    } else if (kind == ORA_NOISE_RADEMACHER) {
        for (int j = 0; j < 4; ++j) out[j] = (x[j] >> 31) ? -1.0 : 1.0;
    } else {
        /* Box-Muller: (u0,u1) -> (r cos 2 pi u1, r sin 2 pi u1), r = sqrt(-2 ln u0);
         * likewise (u2,u3). */
        const double two_pi = 6.283185307179586476925286766559;
        double u0 = ora_uniform(x[0]), u1 = ora_uniform(x[1]);
        double u2 = ora_uniform(x[2]), u3 = ora_uniform(x[3]);
        double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
        out[0] = r0 * cos(two_pi * u1);
        out[1] = r0 * sin(two_pi * u1);
        out[2] = r1 * cos(two_pi * u3);
        out[3] = r1 * sin(two_pi * u3);
    }
}

double ora_noise(uint64_t seed, uint32_t stream, int64_t row, int64_t sweep, int64_t pair, int kind)
{
    double v[4];
    ora_noise_block(seed, stream, (uint32_t)row, (uint32_t)sweep, (uint32_t)(pair / 4), kind, v);
    return v[pair % 4];
}

/* ------------------------------------------------------------------------- */
/* Greedy multicolouring of the symmetrised pattern (edge i-j when c_ij != 0
 * or c_ji != 0 as a stored entry): rows in natural order each take the
 * smallest colour not held by an already coloured neighbour.  The sweep order
 * lists colour 0's rows ascending, then colour 1's, and so on.             */
/* ------------------------------------------------------------------------- */
static void transpose_pattern(int64_t n, const int64_t* rp, const int32_t* col,
                              int64_t** trp_out, int64_t** trow_out, int64_t** tpos_out)
{
    int64_t nnz = rp[n];
    int64_t* trp = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* trow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz ? nnz : 1));
    int64_t* tpos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz ? nnz : 1));
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < nnz; ++e) trp[col[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) trp[i + 1] += trp[i];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int64_t j = col[e];
            int64_t slot = trp[j] + fill[j]++;
            trow[slot] = i;   /* column j holds an entry in row i */
            tpos[slot] = e;   /* ... stored at CSR position e     */
        }
    free(fill);
    *trp_out = trp; *trow_out = trow; *tpos_out = tpos;
}

int ora_greedy_color(int64_t n, const int64_t* rp, const int32_t* col,
                     int32_t* color, int64_t* order, int32_t* ncolors_out)
{
    int64_t *trp, *trow, *tpos;
    transpose_pattern(n, rp, col, &trp, &trow, &tpos);
    int32_t* seen = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 2));
    for (int64_t c = 0; c < n + 2; ++c) seen[c] = -1;
    int32_t ncolors = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int64_t j = col[e];
            if (j < i) seen[color[j]] = (int32_t)i;
        }
        for (int64_t e = trp[i]; e < trp[i + 1]; ++e) {
            int64_t j = trow[e];
            if (j < i) seen[color[j]] = (int32_t)i;
        }
        int32_t c = 0;
        while (seen[c] == (int32_t)i) ++c;
        color[i] = c;
        if (c + 1 > ncolors) ncolors = c + 1;
    }
    int64_t q = 0;
    for (int32_t c = 0; c < ncolors; ++c)
        for (int64_t i = 0; i < n; ++i)
            if (color[i] == c) order[q++] = i;
    *ncolors_out = ncolors;
    free(seen); free(trp); free(trow); free(tpos);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Moment accumulators (eq 1/C and eq tr).                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t groups;        /* G: global pair p is in group p / (pairs_total / G) */
    int64_t pairs_total;   /* P of the whole run                                 */
    int64_t batch_len;     /* samples per time batch                             */
    int64_t n_batches;     /* time batches                                       */
    int64_t samples_done;  /* samples accumulated so far (advanced by the run)   */
    int32_t want_diag;
    int32_t pad_;
    double* diag;          /* [n_batches][G][n] complex, original row order      */
    int64_t nI, nJ;
    const int64_t* bI;     /* requested block rows (original indices)            */
    const int64_t* bJ;     /* requested block columns                            */
    double* block;         /* [n_batches][G][nI][nJ] complex                     */
    int64_t n_entries;
    const int64_t* ei;
    const int64_t* ej;
    double* entries;       /* [n_batches][G][n_entries] complex                  */
    double* trace_series;  /* [max_samples] complex: sum over pairs and rows     */
    int64_t max_samples;
    double* cluster_count; /* [n_batches][G] number of (sample, pair) terms      */
} ora_moments;

enum { ORA_OK = 0, ORA_EINVAL = 1, ORA_DIVERGED = 2, ORA_ESINGULAR = 3 };

/* ------------------------------------------------------------------------- */
/* The sweeps.                                                               */
/* ------------------------------------------------------------------------- */
int ora_sweeps(int64_t n, const int64_t* rp, const int32_t* col, const double* val,
               int is_complex, const int64_t* order,
               uint64_t seed, uint32_t stream, int noise_kind,
               int64_t npairs, const int64_t* pair_ids,
               double* zbuf, double* wbuf, int64_t k0, int64_t nsweeps,
               ora_moments* mom)
{
    cplx* Z = (cplx*)zbuf;  /* Z[i * npairs + p] */
    cplx* W = (cplx*)wbuf;
    int64_t *trp, *trow, *tpos;
    transpose_pattern(n, rp, col, &trp, &trow, &tpos);

    /* Matrix entries as complex numbers (imaginary part 0 for a real matrix). */
    int64_t nnz = rp[n];
    cplx* c = (cplx*)malloc(sizeof(cplx) * (size_t)(nnz ? nnz : 1));
    for (int64_t e = 0; e < nnz; ++e)
        c[e] = is_complex ? CMPLX(val[2 * e], val[2 * e + 1]) : CMPLX(val[e], 0.0);

    /* Per-row constants: inv_i = 1/c_ii and the noise scales a_i, b_i. */
    cplx* inv = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* a = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* b = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    int status = ORA_OK;
    for (int64_t i = 0; i < n && status == ORA_OK; ++i) {
        cplx cii = 0.0;
        int found = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] == i) { cii = c[e]; found = 1; }
        if (!found || cii == 0.0) { status = ORA_ESINGULAR; break; }
        inv[i] = 1.0 / cii;
        if (is_complex) {
            a[i] = 1.0 / csqrt(cii);
            b[i] = conj(a[i]);
        } else {
            double r = creal(cii);
            double s = 1.0 / sqrt(fabs(r));
            a[i] = s;
            b[i] = r > 0 ? s : -s;
        }
    }

    for (int64_t s = 0; s < nsweeps && status == ORA_OK; ++s) {
        int64_t k = k0 + s;
        /* eqs (4) and (5): rows in sweep order, each updated in place, so rows
         * earlier in the order already hold their sweep-k values. */
        for (int64_t q = 0; q < n; ++q) {
            int64_t i = order[q];
            for (int64_t p = 0; p < npairs; ++p) {
                double phi = ora_noise(seed, stream, i, k, pair_ids[p], noise_kind);
                cplx sz = 0.0;
                for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                    int64_t j = col[e];
                    if (j != i) sz += c[e] * Z[j * npairs + p];
                }
                cplx sw = 0.0;
                for (int64_t t = trp[i]; t < trp[i + 1]; ++t) {
                    int64_t j = trow[t];            /* entry c_ji of column i */
                    if (j != i) sw += conj(c[tpos[t]]) * W[j * npairs + p];
                }
                Z[i * npairs + p] = a[i] * phi - inv[i] * sz;
                W[i * npairs + p] = b[i] * phi - conj(inv[i]) * sw;
            }
        }

        /* Divergence: non-finite or runaway state (Sec. 2.2: sp(T), sp(S) >= 1). */
        for (int64_t e = 0; e < n * npairs; ++e) {
            double m = fmax(cabs(Z[e]), cabs(W[e]));
            if (!(m < 1e100)) { status = ORA_DIVERGED; break; }
        }
        if (status != ORA_OK || mom == NULL) continue;

        /* eq (1/C): z w^dagger moments; eq (tr): sum_i z_i conj(w_i). */
        int64_t bidx = mom->samples_done / mom->batch_len;
        if (bidx >= mom->n_batches || mom->samples_done >= mom->max_samples) {
            status = ORA_EINVAL;
            break;
        }
        int64_t gsize = mom->pairs_total / mom->groups;
        for (int64_t p = 0; p < npairs; ++p) {
            int64_t g = pair_ids[p] / gsize;
            int64_t cl = bidx * mom->groups + g;
            if (mom->want_diag) {
                cplx* D = (cplx*)mom->diag + cl * n;
                for (int64_t i = 0; i < n; ++i)
                    D[i] += Z[i * npairs + p] * conj(W[i * npairs + p]);
            }
            if (mom->nI > 0 && mom->nJ > 0) {
                cplx* B = (cplx*)mom->block + cl * mom->nI * mom->nJ;
                for (int64_t r = 0; r < mom->nI; ++r)
                    for (int64_t t = 0; t < mom->nJ; ++t)
                        B[r * mom->nJ + t] += Z[mom->bI[r] * npairs + p] * conj(W[mom->bJ[t] * npairs + p]);
            }
            if (mom->n_entries > 0) {
                cplx* E = (cplx*)mom->entries + cl * mom->n_entries;
                for (int64_t e = 0; e < mom->n_entries; ++e)
                    E[e] += Z[mom->ei[e] * npairs + p] * conj(W[mom->ej[e] * npairs + p]);
            }
            mom->cluster_count[cl] += 1.0;
        }
        if (mom->trace_series) {
            cplx t = 0.0;
            for (int64_t i = 0; i < n; ++i)
                for (int64_t p = 0; p < npairs; ++p)
                    t += Z[i * npairs + p] * conj(W[i * npairs + p]);
            ((cplx*)mom->trace_series)[mom->samples_done] = t;
        }
        mom->samples_done += 1;
    }

    free(c); free(inv); free(a); free(b);
    free(trp); free(trow); free(tpos);
    return status;
}
