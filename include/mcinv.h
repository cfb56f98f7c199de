/*
 * mcinv -- correlated-chains Monte Carlo estimation of entries, the diagonal
 * and the trace of C^-1 for a sparse, possibly non-hermitian matrix C, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Garcia-Cortes & Cabrillo, "A Monte Carlo algorithm for efficient
 * large matrix inversion".  Two vectors z, w are updated row by row with the
 * SAME noise draw phi (Sec. 2, eqs 4 and 5; noise law eqs 5a, 5b):
 *
 *   z_i <- phi_i a_i - (1/c_ii)      [ sum_{j<i} c_ij z_j^(k) + sum_{j>i} c_ij z_j^(k-1) ]
 *   w_i <- phi_i b_i - (1/conj c_ii) [ sum_{j<i} conj(c_ji) w_j^(k) + sum_{j>i} conj(c_ji) w_j^(k-1) ]
 *
 * so that after burn-in E[z w^dagger] = C^-1 (eq 1/C) and E[w^dagger z] =
 * tr C^-1 (eq tr).  The library runs many independent chain pairs at once.
 *
 * Conventions used by every entry point:
 *   - Rows are swept in a greedy multicolour order: a symmetric permutation
 *     P C P^T of the matrix, so one sweep is still eqs 4-5 on the permuted
 *     matrix (Sec. 4 notes that row/column reordering is allowed).  All inputs
 *     and outputs use the caller's ORIGINAL row indices.
 *   - Noise scales satisfy a_i conj(b_i) = 1/c_ii: real c_ii: a = 1/sqrt|c_ii|,
 *     b = sign(c_ii) a; complex: a = 1/sqrt(c_ii) (principal), b = conj(a).
 *   - Noise for (row i, sweep k, pair p) is output (p mod 4) of Philox4x32-10
 *     with key (seed lo, seed hi) and counter (i, k, p div 4, stream_id), p the
 *     global pair index (mcinv_config.pair_offset + the context's own), turned
 *     into N(0,1) by Box-Muller on u = ((x >> 9) + 1/2) 2^-23, or into +-1 (Z2
 *     noise: the sign bit), or 0 (the noiseless Gauss-Seidel of eq 12).
 *   - Complex values are interleaved (re, im) pairs of the stated precision.
 *   - Estimates of entry (i,j) are means of z_i conj(w_j); the trace estimate
 *     is the mean of sum_i z_i conj(w_i) per pair.
 *   - Standard errors: clusters of samples -- chain groups (n_groups >= 16) or
 *     groups x time batches (fewer groups; at most 64 batches, batch length a
 *     power of two) -- with the ratio estimator; the trace uses Geyer's
 *     initial positive sequence on the per-sweep series (Sec. 2.3).
 *
 * Ownership: the caller owns every host pointer it passes; the library copies
 * inputs before returning and writes outputs into caller-allocated memory.  A
 * context owns all of its device memory.  A context is not thread-safe; calls
 * on one context must not overlap.
 *
 * Every function returns an mcinv_status: 0 on success, a negative code on
 * failure (the message is available from mcinv_last_error).
 */
#ifndef MCINV_H
#define MCINV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mcinv_status;

#define MCINV_OK          0
#define MCINV_EINVAL     -1  /* bad argument: shape, order, duplicate, range    */
#define MCINV_ESINGULAR  -2  /* a row has no stored or a zero diagonal (Sec 2.2) */
#define MCINV_ESTATE     -3  /* call out of order (e.g. sample before load_csr)  */
#define MCINV_ENOMEM     -4  /* device or host allocation failed                 */
#define MCINV_EDEVICE    -5  /* a HIP runtime error                              */
#define MCINV_EDIVERGED  -6  /* non-finite or runaway chain state: sp(T) or sp(S)
                                is not below one (Sec. 2.2)                      */
#define MCINV_EINTERNAL  -7  /* unexpected host-side failure (e.g. a worker
                                thread could not start); no exception ever
                                leaves the library                               */

/* Sweep (state) precision. */
#define MCINV_R32   0   /* real, float32 state            */
#define MCINV_R64   1   /* real, float64 state            */
#define MCINV_C64   2   /* complex, 2 x float32 state     */
#define MCINV_C128  3   /* complex, 2 x float64 state     */

/* Noise law (eqs 5a, 5b). */
#define MCINV_NOISE_NORMAL     0
#define MCINV_NOISE_RADEMACHER 1
#define MCINV_NOISE_NONE       2

/* Dense-block moment arithmetic. */
#define MCINV_MOMENTS_FP64   0   /* fp64 products and sums                        */
#define MCINV_MOMENTS_BF16X3 1   /* fp32 state split into bf16 hi+lo, three MFMA
                                    products with fp32 accumulation, fp64 sums   */

/* Requested quantities (bit flags). */
#define MCINV_REQ_DIAG    1u
#define MCINV_REQ_TRACE   2u
#define MCINV_REQ_BLOCK   4u
#define MCINV_REQ_ENTRIES 8u
#define MCINV_REQ_QTRACE  16u  /* tr(Q C^-1) for the Q of mcinv_set_trace_matrix */

typedef struct mcinv_ctx mcinv_ctx;

typedef struct {
    int32_t  device;       /* HIP device ordinal                                     */
    int32_t  sweep_dtype;  /* MCINV_R32 .. MCINV_C128; real dtypes need a real C     */
    int32_t  moments;      /* MCINV_MOMENTS_*                                        */
    int32_t  noise;        /* MCINV_NOISE_*                                          */
    int64_t  n_pairs;      /* P >= 1 independent (z, w) chain pairs                  */
    int32_t  n_groups;     /* G >= 1 chain groups for error estimates; P % G == 0, and
                              for G > 1 the group size P/G is a power of two in
                              [4, 256] or a multiple of 256                           */
    uint32_t stream_id;    /* fourth Philox counter word (distinct problems)        */
    uint64_t seed;         /* Philox key                                             */
    void*    stream;       /* hipStream_t to launch on, or NULL for a library stream */
    int32_t  profile;      /* nonzero: time every sweep launch with HIP events       */
    int32_t  pass_tiles;   /* 256-pair tiles swept through all colours before the
                              next tiles start (cache residency); 0 = automatic   */
    int32_t  xcd_order;    /* sweep workgroup order: 0 natural (round-robin over the
                              8 XCDs), 1 contiguous (tile, row block) ranges per XCD,
                              2 runs of 16 consecutive row blocks per XCD, 3 the
                              pair tiles of a row block one after another;
                              mcinv_tune_launch picks the fastest                 */
    int32_t  hermitian;    /* nonzero: C is hermitian with a positive diagonal
                              (checked by mcinv_load_csr, EINVAL otherwise); then
                              w = z at every step and only z is swept -- the
                              single-draw Gauss-Seidel sampler of eq 2, half the
                              state traffic.  w reads return z; w cannot be written */
    int64_t  pair_offset;  /* global index of this context's first chain pair, a
                              multiple of 4 (0 for a whole run): pair p draws the
                              noise of pair pair_offset + p, so contexts that split
                              one run's pairs between them (one per GPU) reproduce
                              its chains; their moment sums add up to the run's */
    int32_t  stores;       /* sweep state stores: 0 automatic (non-temporal when
                              every colour launch covers all pair tiles, since the
                              new rows are read again only by later launches;
                              temporal in tile passes, whose later colours gather
                              them from the cache), 1 non-temporal, 2 temporal   */
} mcinv_config;

typedef struct {
    int64_t n, nnz, n_pairs, ld;      /* ld: padded pairs per state row           */
    int32_t n_colors, n_groups;
    int64_t sweeps_done, samples_done;
    int64_t batch_len, n_batches;     /* time batching of the error clusters       */
    int64_t offdiag_entries;          /* merged symmetric-pattern entries stored   */
    double  sweep_kernel_ms;          /* profile: summed sweep-kernel time         */
    int64_t sweep_kernel_launches;    /* profile: number of sweep launches timed   */
    double  moment_kernel_ms;         /* profile: block/entry moment kernels       */
    int64_t moment_kernel_launches;
} mcinv_info;

/* Create a context on cfg->device.  *out receives the handle.
 * EINVAL: bad dtype, noise, pairs or group layout.  EDEVICE: HIP failure. */
mcinv_status mcinv_create(const mcinv_config* cfg, mcinv_ctx** out);

/* Release every resource of ctx (NULL is allowed). */
void mcinv_destroy(mcinv_ctx* ctx);

/* Load C (Sec. 2: the matrix to invert) from host CSR arrays.
 * row_ptr int64[n+1] (row_ptr[0] == 0, non-decreasing), col_idx int32[nnz]
 * (strictly increasing within a row, 0 <= col < n), values[nnz] of value_dtype
 * (MCINV_R64 or MCINV_C128, interleaved complex).  Every row must hold a
 * nonzero diagonal entry (ESINGULAR otherwise, Sec. 2.2).  Builds the transpose
 * (eq 5 reads column i of C), the per-row constants in float64 (rounded to the
 * sweep precision), the multicolour order, and uploads everything.  Resets the
 * chain state to z = w = 0 (Algorithm 1, step 1) and clears all moments. */
mcinv_status mcinv_load_csr(mcinv_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col_idx, const void* values, int32_t value_dtype);

/* Choose what to estimate (eq 1/C, eq tr): flags of MCINV_REQ_*; a dense block
 * rows x cols (original indices, any order, may repeat); and a list of entries
 * (entry_i[e], entry_j[e]).  Clears every moment accumulator and the sample
 * count (the chain state is kept).  EINVAL on an index out of range. */
mcinv_status mcinv_set_requested(mcinv_ctx* ctx, uint32_t flags,
                                 const int64_t* block_rows, int64_t n_block_rows,
                                 const int64_t* block_cols, int64_t n_block_cols,
                                 const int64_t* entry_i, const int64_t* entry_j, int64_t n_entries);

/* Run `sweeps` sweeps without accumulating (the burn-in period of Sec. 2.3).
 * EDIVERGED if the state became non-finite or exceeded 1e30 in magnitude. */
mcinv_status mcinv_burn_in(mcinv_ctx* ctx, int64_t sweeps);

/* Run `sweeps` sweeps, each adding one sample per chain pair to every
 * requested moment (eq 1/C, eq tr).  ESTATE before mcinv_set_requested. */
mcinv_status mcinv_sample(mcinv_ctx* ctx, int64_t sweeps);

/* Sample in chunks of check_every sweeps until the largest relative standard
 * error max_i SE_i/|est_i| over the diagonal is <= rel_se, or max_sweeps were
 * run.  With n_groups < 16 the error clusters are time batches, and the stop
 * waits until a batch spans at least 16 sweeps (more than 512 samples) so that
 * batches are close to independent.  Needs MCINV_REQ_DIAG.  *sweeps_done (may
 * be NULL) receives the count, *achieved (may be NULL) the last max relative SE. */
mcinv_status mcinv_sample_until(mcinv_ctx* ctx, double rel_se, int64_t max_sweeps,
                                int64_t check_every, int64_t* sweeps_done, double* achieved);

/* Sample in chunks of check_every sweeps until the trace estimate's standard
 * error (Geyer's initial positive sequence on the per-sweep series, Sec. 2.3)
 * relative to |estimate| is <= rel_se, or max_sweeps -- the stopping rule of
 * the paper's numerical tests, which ran long series.  The error is trusted
 * only once the series holds at least 50 effective samples (S gamma_0 /
 * sigma^2; a shorter series gives too small an error).  Needs MCINV_REQ_TRACE. */
mcinv_status mcinv_sample_until_trace(mcinv_ctx* ctx, double rel_se, int64_t max_sweeps, int64_t check_every,
                                      int64_t* sweeps_done, double* achieved);

/* Estimates and standard errors in original indexing, caller-allocated.
 * quantity: one of MCINV_REQ_DIAG (n values), MCINV_REQ_BLOCK (rows x cols,
 * row-major), MCINV_REQ_ENTRIES (n_entries), MCINV_REQ_TRACE or MCINV_REQ_QTRACE (1 value).
 * est receives 1 double per value for a real C, 2 (re, im) for a complex C;
 * stderr_ receives 1 double per value (sqrt(SE_re^2 + SE_im^2)); either may be
 * NULL.  capacity = number of values the arrays can hold (EINVAL if short).
 * SE is NaN while fewer than two clusters hold samples. */
mcinv_status mcinv_read_estimates(mcinv_ctx* ctx, uint32_t quantity, double* est,
                                  double* stderr_, int64_t capacity);

/* The quantities the paper's Tables 2, 4 and 5 report for a trace (Sec. 2.3,
 * Sec. 3): Geyer's initial positive sequence on the per-sweep series x_k =
 * (1/P) sum_p t_p^(k) of MCINV_REQ_TRACE or MCINV_REQ_QTRACE.  stats[9]:
 * mean (re, im; im 0 for a real C), gamma_0 (the series' variance, summed
 * over re and im), sigma^2 = -gamma_0 + 2 sum_m Gamma_m, the effective length
 * S gamma_0 / sigma^2, the standard error sqrt(sigma^2 / S), S, and gamma_0
 * of the real and of the imaginary part separately.  The
 * series averages P chain pairs, so gamma_0 P and (effective length) P are
 * the single-pair figures the tables print.  ESTATE: not requested or no
 * samples. */
mcinv_status mcinv_read_trace_stats(mcinv_ctx* ctx, uint32_t quantity, double* stats);

/* Copy chain state z (which = 0) or w (which = 1) to host as [n][P] in the
 * sweep precision, original row order.  bytes must be >= n * P * elem size. */
mcinv_status mcinv_read_state(mcinv_ctx* ctx, int32_t which, void* host, int64_t bytes);

/* Overwrite chain state z or w from a host [n][P] array (sweep precision,
 * original order), e.g. to start from other initial values (Algorithm 1). */
mcinv_status mcinv_write_state(mcinv_ctx* ctx, int32_t which, const void* host, int64_t bytes);

/* The sweep order: perm[q] = original row swept at position q (int64[n]);
 * color_of_row[i] = colour of original row i (int32[n]).  Either may be NULL. */
mcinv_status mcinv_get_permutation(mcinv_ctx* ctx, int64_t* perm, int32_t* color_of_row);

/* Burn-in by coupling (Sec. 2.3, Algorithm 1 steps 1-5): a second path per
 * chain started at x*_i = i (1-based original index) and driven by the same
 * noise is run until both coupled differences, max_i |z_i - z*_i| and
 * max_i |w_i - w*_i|, are below tol (the paper uses 5e-5).  By eq 12 the
 * difference of two such paths is the noiseless Gauss-Seidel iteration on
 * C d = 0 (z) and C^dagger d = 0 (w), identical for every chain pair, so the
 * library runs that one iteration (in the sweep precision), checks it after
 * every sweep, and advances the chains by the same number N of noisy sweeps:
 * the chains end exactly as after mcinv_burn_in(ctx, N).  The iteration runs
 * on a stream of the library's own, ahead of the chains; chain sweep k is
 * issued on the context's stream once the difference shows N >= k, so the two
 * overlap.  Stops at max_sweeps if the tolerance is not reached (*diff_z /
 * *diff_w tell).  EDIVERGED when the difference becomes non-finite (the chain
 * sweeps issued until then have run).  Outputs may be NULL. */
mcinv_status mcinv_burn_in_coupled(mcinv_ctx* ctx, double tol, int64_t max_sweeps, int64_t* sweeps_done,
                                   double* diff_z, double* diff_w);

/* Time sweeps_per_trial burn-in sweeps (after one warm-up sweep) under each
 * workgroup order (mcinv_config.xcd_order 0 .. 3) and keep the fastest.  The
 * chains advance as in mcinv_burn_in (4 + 4 sweeps_per_trial sweeps; the
 * order never changes the arithmetic, so results do not depend on it).
 * ms_orders[4] (may be NULL): ms per sweep of each order; xcd_order may be NULL. */
mcinv_status mcinv_tune_launch(mcinv_ctx* ctx, int32_t sweeps_per_trial, int32_t* xcd_order, double* ms_orders);

/* Noiseless sweeps from x_i = i (Algorithm 1's second start) on C x = 0 and
 * C^dagger y = 0: the Gauss-Seidel iterations eq 12 shows the chain
 * difference obeys.  Returns the observed contraction rates, which tend to
 * sp(T) and sp(S) (Sec. 2.3).  Does not touch the chain state.  iters >= 2. */
mcinv_status mcinv_check_convergence(mcinv_ctx* ctx, int64_t iters, double* rho_T, double* rho_S);

/* A sparse Q for tr(Q C^-1) = E[w^dagger Q z] (eq tr; Algorithm 1, step 8
 * accumulates this product per sweep): n x n CSR in original indices,
 * values of value_dtype (MCINV_R64, or MCINV_C128 with a complex sweep
 * dtype), any column order.  Request it with MCINV_REQ_QTRACE; the estimate
 * and its Geyer standard error are read with quantity MCINV_REQ_QTRACE and
 * mcinv_sample_until_trace stops on it when requested.  Kept until the next
 * mcinv_load_csr.  ESTATE while MCINV_REQ_QTRACE is requested. */
mcinv_status mcinv_set_trace_matrix(mcinv_ctx* ctx, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                                    const void* values, int32_t value_dtype);

/* Checkpoint / resume.  mcinv_save writes the chain state, the requested
 * set, every moment accumulator, the trace series and the counters to a file;
 * mcinv_restore reads it into a context created with the same configuration
 * (pairs, groups, dtype, seed, stream_id, noise, hermitian) on which the same
 * matrix has been loaded (the colour order is fingerprinted; the values are
 * the caller's responsibility) and, if the checkpoint requested
 * MCINV_REQ_QTRACE, the same Q set.  The restored context continues exactly
 * as the saved one would (same noise counters, same sums).  EINVAL on a
 * mismatch or an unreadable file; a file whose counts or size do not match
 * its header (damaged, truncated) is rejected before the context changes. */
mcinv_status mcinv_save(mcinv_ctx* ctx, const char* path);
mcinv_status mcinv_restore(mcinv_ctx* ctx, const char* path);

/* Restrict the stop check of mcinv_sample_until (max SE/|est| of the
 * diagonal) to the given original rows; count 0 restores every row.  The
 * estimates of all rows are still computed.  Cleared by mcinv_load_csr. */
mcinv_status mcinv_set_stop_rows(mcinv_ctx* ctx, const int64_t* rows, int64_t count);

/* Sizes, counters and (when profiling) kernel times. */
mcinv_status mcinv_get_info(mcinv_ctx* ctx, mcinv_info* out);

/* Zero the profiling counters of mcinv_get_info. */
mcinv_status mcinv_reset_profile(mcinv_ctx* ctx);

/* Noise values phi(row[t], sweep[t], pair[t]) as the sweep kernels draw them,
 * generated on the device in the given precision (MCINV_R32 or MCINV_R64) and
 * copied to out[count] (double).  For checking the generator. */
mcinv_status mcinv_noise_values(int32_t device, uint64_t seed, uint32_t stream_id,
                                int32_t noise, int32_t dtype, int64_t count,
                                const int64_t* row, const int64_t* sweep, const int64_t* pair,
                                double* out);

/* Message of the last failing call on ctx (or of the last failing call that
 * had no context, when ctx is NULL). */
const char* mcinv_last_error(const mcinv_ctx* ctx);

/* ------------------------------------------------------------------------ */
/* Batched form: many real matrices of uneven order, each with its own n_pairs
 * chain pairs (fp32 sweeps, eqs 4-5), all swept together by one graph launch
 * per call (a persistent kernel, or one kernel per colour phase; see the
 * schedules below).  Matrix m is prepared exactly as
 * a single-matrix context would prepare it and draws its noise with
 * stream_id = m, so its chains are bit-identical to a single-matrix context
 * with the same seed and stream_id = m.  Moments: the diagonal (fp64 sums,
 * groups as in a single context) and one dense block per matrix whose
 * products run on the matrix cores as bf16x3 (hi*hi + hi*lo + lo*hi, fp32
 * accumulation over the pairs, fp64 sums); block standard errors come from 16
 * time batches of length ceil(expected_samples / 16).                        */
typedef struct mcinv_batch mcinv_batch;

/* Batched schedules.  PERSISTENT: one launch runs all sweeps of a call; work
 * items (sweep, colour, matrix, row chunk) are taken in order from a device
 * queue and wait on per-matrix completion counters (agent-scope release /
 * acquire).  PHASED: per sweep one launch per colour across all matrices and
 * one for the block moments, the whole call captured as one HIP graph and
 * replayed with a single graph launch; kernel boundaries order the phases. */
#define MCINV_SCHEDULE_PHASED     0
#define MCINV_SCHEDULE_PERSISTENT 1

typedef struct {
    int32_t  device;
    int32_t  noise;          /* MCINV_NOISE_*                                    */
    int64_t  n_pairs;        /* P per matrix: 16, 32, 64, 128 or 256             */
    int32_t  n_groups;       /* G: P/G a power of two >= 4                       */
    int32_t  rows_per_item;  /* rows per work item (0: 64; see autotune)         */
    int32_t  grab;           /* persistent schedule: items per queue access (0: 4) */
    int32_t  schedule;       /* MCINV_SCHEDULE_PHASED or MCINV_SCHEDULE_PERSISTENT */
    uint64_t seed;           /* Philox key (shared by all matrices)             */
    void*    stream;         /* hipStream_t or NULL for a library stream         */
} mcinv_batch_config;

typedef struct {
    int64_t n_matrices, n_rows, nnz, n_pairs;
    int32_t n_groups, max_colors, rows_per_item, grab, grid, schedule;
    int64_t items_per_sweep, sweeps_done, samples_done;
    double  last_call_ms;    /* device time of the last burn_in / sample call   */
} mcinv_batch_info;

/* Create an empty batch of n_matrices matrices.  EINVAL on a bad layout. */
mcinv_status mcinv_batch_create(const mcinv_batch_config* cfg, int64_t n_matrices, mcinv_batch** out);
void mcinv_batch_destroy(mcinv_batch* b);

/* Load matrix m (real, float64 values; CSR rules as mcinv_load_csr).  All
 * matrices must be loaded before the first other call; the batch is then
 * fixed.  ESINGULAR / EINVAL as mcinv_load_csr. */
mcinv_status mcinv_batch_load_csr(mcinv_batch* b, int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                  const int32_t* col_idx, const double* values);

/* flags: MCINV_REQ_DIAG and/or MCINV_REQ_BLOCK.  block_dim (1..128): each
 * matrix's block is its last block_dim rows x columns unless set with
 * mcinv_batch_set_block.  expected_samples sets the block time-batch length.
 * Clears the moments and the sample counts, and makes every matrix active
 * again (see mcinv_batch_sample_until_each). */
mcinv_status mcinv_batch_set_requested(mcinv_batch* b, uint32_t flags, int32_t block_dim, int64_t expected_samples);

/* Block rows and columns of matrix m (block_dim original indices each). */
mcinv_status mcinv_batch_set_block(mcinv_batch* b, int64_t m, const int64_t* rows, const int64_t* cols);

/* Burn-in / sampling sweeps of every active matrix (one persistent launch per
 * call, split only beyond 2^30 work items).  EDIVERGED as mcinv_burn_in;
 * EDEVICE if a dependency wait inside the launch exceeded its bound. */
mcinv_status mcinv_batch_burn_in(mcinv_batch* b, int64_t sweeps);
mcinv_status mcinv_batch_sample(mcinv_batch* b, int64_t sweeps);

/* Burn-in by coupling for every matrix (as mcinv_burn_in_coupled): the
 * noiseless difference iteration of eq 12 runs for all matrices together
 * until the largest coupled difference over all matrices is below tol, then
 * every matrix advances by that common number N of sweeps (a matrix whose own
 * coupling converged earlier burns in longer, which only lowers its bias).
 * *max_diff: the largest difference at N.  Outputs may be NULL. */
mcinv_status mcinv_batch_burn_in_coupled(mcinv_batch* b, double tol, int64_t max_sweeps, int64_t* sweeps_done,
                                         double* max_diff);

/* Sample in chunks until max over all matrices and rows of SE/|est| of the
 * diagonal is <= rel_se (or max_sweeps).  With fewer than 16 chain groups the
 * error clusters are time batches of ceil(expected_samples / 16) sweeps; both
 * stopping rules return EINVAL when those are shorter than 16 sweeps (short
 * batches of an autocorrelated chain understate the SE). */
mcinv_status mcinv_batch_sample_until(mcinv_batch* b, double rel_se, int64_t max_sweeps, int64_t check_every,
                                      int64_t* sweeps_done, double* achieved);

/* Per-matrix stopping rule: sample in chunks of check_every sweeps; after each
 * chunk, every active matrix whose max over rows of SE/|est| (diagonal) is
 * <= rel_se stops -- it gets no further sweeps, so its chains, moments and
 * sample count stay as they were (each matrix ends where mcinv_sample_until
 * would have ended it alone, given the same burn-in).  Ends when no matrix is
 * active or after max_sweeps.  *sweeps_done: sweeps of the longest-running
 * matrix; *achieved: max over all matrices of their last checked value.
 * Later burn_in / sample calls sweep only the active matrices;
 * mcinv_batch_set_requested reactivates all.  Outputs may be NULL. */
mcinv_status mcinv_batch_sample_until_each(mcinv_batch* b, double rel_se, int64_t max_sweeps, int64_t check_every,
                                           int64_t* sweeps_done, double* achieved);

/* Per matrix: samples accumulated (int64_t[n_matrices]) and whether it is
 * still active (uint8_t[n_matrices], 1 = active).  Either may be NULL. */
mcinv_status mcinv_batch_matrix_samples(mcinv_batch* b, int64_t* samples, uint8_t* active);

/* Estimates of matrix m: MCINV_REQ_DIAG (n values, original order) or
 * MCINV_REQ_BLOCK (block_dim^2, row-major); est and stderr_ as
 * mcinv_read_estimates (real). */
mcinv_status mcinv_batch_read_estimates(mcinv_batch* b, int64_t m, uint32_t quantity, double* est,
                                        double* stderr_, int64_t capacity);

/* Training labels of the learned surrogate for matrix m: the sampler's
 * diagonal estimate (eq 1/C) scaled to the surrogate's target,
 * y[i] = c_ii (C^-1)_ii, and its standard error y_se[i] = |c_ii| SE_i, both
 * float64[n] in original row order (capacity >= n).  Errors as
 * mcinv_batch_read_estimates(MCINV_REQ_DIAG). */
mcinv_status mcinv_batch_read_labels(mcinv_batch* b, int64_t m, double* y, double* y_se, int64_t capacity);

/* Chain state of matrix m, [n][P] fp32, original row order. */
mcinv_status mcinv_batch_read_state(mcinv_batch* b, int64_t m, int32_t which, float* host, int64_t bytes);

/* Time every (schedule, rows per item, items per grab) candidate on
 * sweeps_per_trial burn-in sweeps (plus one warm-up each; the chains advance
 * as in burn-in, and the schedule never changes the chains) and keep the
 * fastest; a schedule whose first candidate takes over twice the best time so
 * far is not explored further.  Any output pointer may be NULL. */
mcinv_status mcinv_batch_autotune(mcinv_batch* b, int32_t sweeps_per_trial, int32_t* schedule,
                                  int32_t* rows_per_item, int32_t* grab, double* ms_per_sweep);

mcinv_status mcinv_batch_get_info(mcinv_batch* b, mcinv_batch_info* out);
const char* mcinv_batch_last_error(const mcinv_batch* b);

/* ------------------------------------------------------------------------ */
/* Learned surrogate of the diagonal.  Writing C = D (I + M), M = D^-1 R with
 * R the off-diagonal part, the series C^-1 = sum_k (-M)^k D^-1 (it converges
 * under the dominance that Sec. 2.3 needs for the sampler) gives
 *     y_i = c_ii (C^-1)_ii = 1 + (M^2)_ii - (M^3)_ii + ...
 * The surrogate predicts y_i from local terms of that series and statistics of
 * row i's neighbourhood; the sampler's estimates (eq 1/C) are its labels, and
 * a gate sends the rows whose validated error is too large back to the
 * sampler.                                                                   */

#define MCINV_N_FEATURES 32

/* Features of every row of a real matrix (CSR rules as mcinv_load_csr,
 * float64 values), out[n][32] float32 in the caller's row order, computed in
 * fp64 on the device.  Feature k of row i (m_ij = c_ij / c_ii; "neighbours"
 * are the j != i with c_ij or c_ji stored; r_j = row abs sum / |c_jj|):
 *   0 log|c_ii|                       1 sum_j |c_ij| / |c_ii| (= r_i)
 *   2 sum_j |c_ji| / |c_ii|           3, 4 row / column off-diagonal count / 8
 *   5 (M^2)_ii                        6 (M^3)_ii
 *   7 sum_j |m_ij| |m_ji|             8 sum_j m_ij^2
 *   9 sum_j c_ij / c_ii              10 sum_j c_ji / c_ii
 *  11-14 mean, max, min, std of the neighbours' r_j
 *  15-17 mean, max, min of log|c_jj| - log|c_ii|;  18 std of log|c_jj|
 *  19, 20 mean, max of the neighbours' (M^2)_jj
 *  21, 22 mean, max of the neighbours' feature 2;  23 mean of their (M^3)_jj
 *  24 neighbour count / 8     25 1 + (M^2)_ii     26 1 + (M^2)_ii - (M^3)_ii
 *  27 r_i^2    28 ((M^2)_ii)^2    29 (M^2)_ii r_i    30 sum_j r_j^2 / 8    31 1
 * Statistics over an empty neighbourhood are 0.  ESINGULAR / EINVAL as
 * mcinv_load_csr; the message is mcinv_last_error(NULL). */
mcinv_status mcinv_features(int32_t device, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                            const double* values, float* out);

/* mcinv_features for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same features, bit for bit, from the same kernels, but every array is
 * DEVICE memory the caller owns -- row_ptr int64[n+1], col_idx int32[nnz],
 * values float64[nnz] in, out float32[n][32] -- and the scratch buffers
 * (column counts and pointers, the transposed entries, the merged neighbour
 * lists, the per-row terms) come from a fixed 32 MiB device array of the
 * library, which each GPU keeps for the life of the process.  Limits: 1 <= n
 * <= 32768 and n <= nnz <= 262144, else EINVAL.  The CSR rules of
 * mcinv_load_csr are checked on the device (EINVAL for a pattern error,
 * ESINGULAR for a missing or zero diagonal; the message, from
 * mcinv_last_error(NULL), names the kind of error but not the row).  Runs on
 * `stream` (a hipStream_t, NULL for the default stream) and synchronises it
 * before returning.  No device or host memory is allocated on success (an
 * error message may allocate).  Calls on one GPU share its scratch array, so
 * calls that overlap on one GPU (from several host threads) race. */
mcinv_status mcinv_features_noalloc(int32_t device, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                    const int32_t* col_idx, const double* values, float* out, void* stream);

/* The network: 32 -> 128 -> 128 -> 1, GELU (erf form) after the two hidden
 * layers.  Parameters, float32, in this order (20865 values):
 *   W1[32][128] (input-major), b1[128], W2[128][128] (input-major), b2[128],
 *   w3[128], b3.
 * Features are normalised as (x - mean) * inv_std before the first layer.
 * Products run on the matrix cores with bf16 operands (round to nearest even:
 * the normalised features, W1, W2, the first hidden activations and both
 * hidden layers' deltas) and fp32 accumulation; everything else is fp32, the
 * GELU through an erf approximation with absolute error at most 1.5e-7.
 * Training minimises sum_r w_r (out_r - y_r)^2 / R over batches of R rows
 * with Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on fp32
 * master weights; every sum runs in a fixed order, so training is
 * reproducible on one device.  Zero-initialised parameters until set. */
#define MCINV_MLP_PARAMS 20865
typedef struct mcinv_mlp mcinv_mlp;

mcinv_status mcinv_mlp_create(int32_t device, mcinv_mlp** out);
void mcinv_mlp_destroy(mcinv_mlp* m);
/* Set (and reset Adam's moments and step count) / read the parameters. */
mcinv_status mcinv_mlp_set_params(mcinv_mlp* m, const float* params);
mcinv_status mcinv_mlp_get_params(mcinv_mlp* m, float* params);
/* mean[32], inv_std[32]: the feature normalisation (default 0 and 1). */
mcinv_status mcinv_mlp_set_normalization(mcinv_mlp* m, const float* mean, const float* inv_std);
/* Training rows: X[N][32] raw features, labels y[N], row weights w[N]
 * (copied to the device; replaces earlier data). */
mcinv_status mcinv_mlp_set_data(mcinv_mlp* m, const float* X, const float* y, const float* w, int64_t N);
/* Set the normalisation to the training data's column means and inverse
 * standard deviations (population, fp64; 1 for a constant column) and return
 * them (either pointer may be NULL). */
mcinv_status mcinv_mlp_fit_normalization(mcinv_mlp* m, float* mean, float* inv_std);
/* Row weights of the loss from the labels' standard errors:
 * w_i = 1 / (se_i^2 + eps), scaled to mean 1.  Host code. */
mcinv_status mcinv_mlp_label_weights(int64_t N, const double* y_se, double eps, float* w);
/* Gradient of the loss over the given training rows (nrows a positive
 * multiple of 64, indices in [0, N)) at the current parameters, grads[20865]
 * in parameter order, and the loss.  Does not change the parameters. */
mcinv_status mcinv_mlp_gradients(mcinv_mlp* m, const int64_t* rows, int32_t nrows, float* grads, float* loss);
/* steps Adam steps with learning rate lr.  Step t (counted from the last
 * set_params, starting at 1) trains on the rows floor(x N / 2^64), x = (o0 << 32)
 * | o1 of the Philox4x32-10 block with key (seed lo, seed hi) and counter (r,
 * t, 0x5EED, 0xA11CE), r = 0..batch_rows-1.  batch_rows: a multiple of 64 up
 * to 2^20.  loss_history (may be NULL): steps values, the loss before each step. */
mcinv_status mcinv_mlp_train(mcinv_mlp* m, int64_t steps, int32_t batch_rows, float lr, uint64_t seed,
                             float* loss_history);
/* Predictions out[N] for raw features X[N][32] (host arrays). */
mcinv_status mcinv_mlp_predict(mcinv_mlp* m, const float* X, int64_t N, float* out);
const char* mcinv_mlp_last_error(const mcinv_mlp* m);

/* The gate: which rows take the network's prediction and which go back to
 * the sampler.  Validation rows (features X[N][32], predictions, sampler
 * labels y and their standard errors) are binned on two features, each by its
 * quantile edges: the sorted values at floor(k N / bins), k = 1..bins-1, and a
 * value's bin is the number of edges <= it.  A bin's validated relative error
 * is sqrt(max(sum r^2 - sum s^2, 0) / count), r = (pred - y)/y, s = se/y (the
 * observed spread less what the label noise explains).  With ucb_z > 0 the
 * error compared with tol is instead an upper confidence bound for it,
 * sqrt(max(sum r^2 - sum s^2, 0) / q), where q is the lower quantile of a
 * chi-square with count degrees of freedom at standard normal quantile -ucb_z
 * (Wilson-Hilferty: q = k (1 - 2/(9k) - ucb_z sqrt(2/(9k)))^3, k = count;
 * ucb_z = 1.645: one-sided 95%), so a bin with few rows needs a smaller
 * observed error.  The bin needs the sampler when it holds fewer than
 * min_rows rows or that error exceeds tol.  Host code, float64. */
typedef struct {
    int32_t feature_a, feature_b;  /* binning features, 0..31                    */
    int32_t bins;                  /* bins per feature, 1..256                    */
    int32_t min_rows;              /* fewer validation rows in a bin: sampler     */
    double  tol;                   /* largest accepted relative error (e.g. 0.01) */
    double  ucb_z;                 /* 0: point estimate; > 0: upper bound at that
                                      normal quantile (see above)                 */
} mcinv_gate_config;
typedef struct mcinv_gate mcinv_gate;

/* EINVAL: bad configuration, a non-finite binning feature, a zero or
 * non-finite label. */
mcinv_status mcinv_gate_fit(const mcinv_gate_config* cfg, int64_t N, const float* X, const double* pred,
                            const double* y, const double* y_se, mcinv_gate** out);
/* fallback[i] = 1 when row i's bin needs the sampler, or a binning feature is
 * NaN or lies outside the [min, max] range of the validation rows (the outer
 * bins are open-ended, so such a row has no validated error). */
mcinv_status mcinv_gate_apply(const mcinv_gate* g, int64_t N, const float* X, uint8_t* fallback);
/* edges_a, edges_b [bins-1]; bin_err, bin_count, bin_fallback [bins * bins],
 * bin (a, b) at a * bins + b.  bin_err is the value compared with tol (the
 * upper bound when ucb_z > 0; +inf for an empty bin).  range[4]: min and max
 * of feature_a, then of feature_b, over the validation rows.  Any may be
 * NULL. */
mcinv_status mcinv_gate_read(const mcinv_gate* g, double* edges_a, double* edges_b, double* bin_err,
                             int64_t* bin_count, uint8_t* bin_fallback, double* range);
void mcinv_gate_destroy(mcinv_gate* g);

/* The surrogate's whole estimate of one matrix in one call: the features of
 * the real CSR matrix (rules of mcinv_features) are computed on the network's
 * device and fed to the network there, so only the predictions and the gate's
 * two binning features cross to the host.  est[n] = the surrogate's estimate
 * of (C^-1)_ii: the network's output (c_ii (C^-1)_ii, as mcinv_mlp_predict on
 * mcinv_features' output) divided by c_ii in fp64; fallback[n] = the gate's
 * decision per row (as mcinv_gate_apply on those features), or 1 where the
 * network's output is not finite: 1 where est must come from the sampler
 * instead.  Both caller-allocated.  ESINGULAR / EINVAL
 * as mcinv_features; the message is available from mcinv_mlp_last_error(m). */
mcinv_status mcinv_mlp_estimate_matrix(mcinv_mlp* m, const mcinv_gate* g, int64_t n, int64_t nnz,
                                       const int64_t* row_ptr, const int32_t* col_idx, const double* values,
                                       double* est, uint8_t* fallback);
const char* mcinv_gate_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCINV_H */
