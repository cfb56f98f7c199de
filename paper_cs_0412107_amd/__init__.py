"""mcinv on MI355X: correlated-chains Monte Carlo estimation of entries, the
diagonal and the trace of C^-1 (Garcia-Cortes & Cabrillo), hand-written HIP
kernels for gfx950 behind the C-ABI of ``include/mcinv.h``.

``Sampler`` is a thin object wrapper over the ``mcinv_*`` binding; PyTorch is
used only (optionally) to hand the library its current HIP stream.
"""

from ._binding import *  # noqa: F401,F403
from ._binding import (DTYPES, MCINV_MOMENTS_BF16X3, MCINV_MOMENTS_FP64, MCINV_NOISE_NORMAL,
                       MCINV_REQ_BLOCK, MCINV_REQ_DIAG, MCINV_REQ_ENTRIES, MCINV_REQ_TRACE, McinvError, lib,
                       mcinv_burn_in, mcinv_check_convergence, mcinv_create, mcinv_destroy, mcinv_get_info,
                       mcinv_get_permutation, mcinv_load_csr, mcinv_read_estimates, mcinv_read_state,
                       mcinv_reset_profile, mcinv_sample, mcinv_sample_until, mcinv_set_requested,
                       mcinv_write_state)

from ._binding import (mcinv_batch_autotune, mcinv_batch_burn_in, mcinv_batch_create, mcinv_batch_destroy,
                       mcinv_batch_get_info, mcinv_batch_load_csr, mcinv_batch_read_estimates,
                       mcinv_batch_read_labels,
                       mcinv_batch_read_state, mcinv_batch_sample, mcinv_batch_sample_until,
                       mcinv_batch_set_block, mcinv_batch_set_requested)

__all__ = ["Sampler", "BatchSampler", "McinvError", "lib"]


def torch_stream():
    """The current torch HIP stream handle (or None when torch has no GPU)."""
    try:
        import torch
    except ImportError:
        return None
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream().cuda_stream


class Sampler:
    """One context: a matrix, its chain pairs and the requested moments.

    ``matrix``: CSR with ``n``, ``row_ptr``, ``col``, ``val`` (float64 or
    complex128 values); ``pairs`` independent (z, w) chain pairs in ``groups``
    error groups; ``dtype`` the sweep precision ("f32", "f64", "c64", "c128");
    ``moments="bf16x3"`` puts dense blocks on the matrix cores (fp32 sweeps).
    All row indices are the matrix's own.  Usable as a context manager."""

    def __init__(self, matrix, pairs, groups=1, dtype="f32", seed=0, noise=MCINV_NOISE_NORMAL,
                 moments="fp64", device=0, stream_id=0, use_torch_stream=False, profile=False, pass_tiles=0,
                 hermitian=False, xcd_order=0, pair_offset=0, stores=0):
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        self.is_complex = self.dtype in (DTYPES["c64"], DTYPES["c128"])
        mom = MCINV_MOMENTS_BF16X3 if moments == "bf16x3" else MCINV_MOMENTS_FP64
        stream = torch_stream() if use_torch_stream else None
        self.ctx = mcinv_create(device=device, sweep_dtype=self.dtype, moments=mom, noise=noise,
                                n_pairs=pairs, n_groups=groups, stream_id=stream_id, seed=seed,
                                stream=stream, profile=profile, pass_tiles=pass_tiles, hermitian=hermitian,
                                xcd_order=xcd_order, pair_offset=pair_offset, stores=stores)
        self.n = matrix.n
        self.P = pairs
        self.nI = self.nJ = self.ne = 0
        try:
            mcinv_load_csr(self.ctx, matrix.n, matrix.nnz, matrix.row_ptr, matrix.col, matrix.val)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "ctx", None) is not None:
            mcinv_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_trace_matrix(self, Q):
        """Q (CSR with row_ptr, col, val, or a scipy sparse matrix) for tr(Q C^-1)."""
        from ._binding import mcinv_set_trace_matrix
        if hasattr(Q, "tocsr"):
            Q = Q.tocsr()
            rp, ci, v = Q.indptr, Q.indices, Q.data
        else:
            rp, ci, v = Q.row_ptr, Q.col, Q.val
        mcinv_set_trace_matrix(self.ctx, self.n, rp, ci, v)

    def qtrace(self):
        """(estimate, SE) of tr(Q C^-1) for the Q of ``set_trace_matrix``."""
        from ._binding import MCINV_REQ_QTRACE
        est, se = mcinv_read_estimates(self.ctx, MCINV_REQ_QTRACE, 1, self.is_complex)
        return est[0], se[0]

    def request(self, diag=True, trace=True, block_rows=None, block_cols=None, entries=None, qtrace=False):
        """Choose the moments to accumulate (clears earlier ones): the diagonal,
        the trace, the dense block rows x cols, entries [(i, j), ...], tr(Q C^-1)."""
        from ._binding import MCINV_REQ_QTRACE
        flags = (MCINV_REQ_DIAG if diag else 0) | (MCINV_REQ_TRACE if trace else 0) | \
            (MCINV_REQ_QTRACE if qtrace else 0)
        ei = ej = None
        if block_rows is not None and block_cols is not None and len(block_rows) and len(block_cols):
            flags |= MCINV_REQ_BLOCK
            self.nI, self.nJ = len(block_rows), len(block_cols)
        if entries is not None and len(entries):
            import numpy as np
            e = np.asarray(entries, dtype=np.int64).reshape(-1, 2)
            ei, ej = e[:, 0], e[:, 1]
            flags |= MCINV_REQ_ENTRIES
            self.ne = e.shape[0]
        mcinv_set_requested(self.ctx, flags, block_rows, block_cols, ei, ej)

    def burn_in(self, sweeps):
        """Sweeps whose samples are discarded."""
        mcinv_burn_in(self.ctx, sweeps)

    def burn_in_coupled(self, tol=5e-5, max_sweeps=10000):
        """Burn in until the coupled paths agree to tol; returns (sweeps, diff_z, diff_w)."""
        from ._binding import mcinv_burn_in_coupled
        return mcinv_burn_in_coupled(self.ctx, tol, max_sweeps)

    def sample(self, sweeps):
        """Sampling sweeps: one sample per pair each."""
        mcinv_sample(self.ctx, sweeps)

    def sample_until(self, rel_se, max_sweeps, check_every=10):
        """Sample until max_i SE_i / |est_i| <= rel_se on the diagonal; returns (sweeps, achieved)."""
        return mcinv_sample_until(self.ctx, rel_se, max_sweeps, check_every)

    def sample_until_trace(self, rel_se, max_sweeps, check_every=20):
        """Sample until the trace's Geyer SE / |estimate| <= rel_se; returns (sweeps, achieved)."""
        from ._binding import mcinv_sample_until_trace
        return mcinv_sample_until_trace(self.ctx, rel_se, max_sweeps, check_every)

    def diag(self):
        """(estimates, SEs) of (C^-1)_ii."""
        return mcinv_read_estimates(self.ctx, MCINV_REQ_DIAG, self.n, self.is_complex)

    def block(self):
        """(estimates, SEs) of the requested block, rows x cols."""
        est, se = mcinv_read_estimates(self.ctx, MCINV_REQ_BLOCK, self.nI * self.nJ, self.is_complex)
        return est.reshape(self.nI, self.nJ), se.reshape(self.nI, self.nJ)

    def entries(self):
        """(estimates, SEs) of the requested entries."""
        return mcinv_read_estimates(self.ctx, MCINV_REQ_ENTRIES, self.ne, self.is_complex)

    def trace(self):
        """(estimate, Geyer SE) of tr(C^-1)."""
        est, se = mcinv_read_estimates(self.ctx, MCINV_REQ_TRACE, 1, self.is_complex)
        return est[0], se[0]

    def trace_stats(self, q=False):
        """Geyer statistics of the trace series (tr C^-1, or tr(Q C^-1) with q):
        mean, variance, sigma2, effective length, SE, samples."""
        from ._binding import MCINV_REQ_QTRACE, MCINV_REQ_TRACE, mcinv_read_trace_stats
        return mcinv_read_trace_stats(self.ctx, MCINV_REQ_QTRACE if q else MCINV_REQ_TRACE)

    def state(self, which):
        """Chain state z (which=0) or w (1), [n][pairs], original row order."""
        return mcinv_read_state(self.ctx, which, self.n, self.P, self.dtype)

    def set_state(self, which, values):
        mcinv_write_state(self.ctx, which, values, self.dtype)

    def permutation(self):
        """(position order, colour of each row) of the multicolour sweep."""
        return mcinv_get_permutation(self.ctx, self.n)

    def save(self, path):
        from ._binding import mcinv_save
        mcinv_save(self.ctx, path)

    def restore(self, path):
        """Load a checkpoint.  Call ``request`` with the checkpoint's arguments
        first so that this wrapper knows the block and entry sizes."""
        from ._binding import mcinv_restore
        mcinv_restore(self.ctx, path)

    def set_stop_rows(self, rows=None):
        """Restrict ``sample_until``'s stop check to these original rows (None: all)."""
        from ._binding import mcinv_set_stop_rows
        mcinv_set_stop_rows(self.ctx, rows)

    def tune_launch(self, sweeps_per_trial=2):
        """Pick the fastest sweep workgroup order; returns (order, ms per sweep of orders 0, 1, 2)."""
        from ._binding import mcinv_tune_launch
        return mcinv_tune_launch(self.ctx, sweeps_per_trial)

    def check_convergence(self, iters=200):
        """Contraction rates of the noiseless iteration (eq 12): estimates of sp(T), sp(S)."""
        return mcinv_check_convergence(self.ctx, iters)

    def info(self):
        return mcinv_get_info(self.ctx)

    def reset_profile(self):
        mcinv_reset_profile(self.ctx)


class BatchSampler:
    """The batched form: many real matrices, ``pairs`` chain pairs each, fp32
    sweeps in one persistent launch per call."""

    def __init__(self, matrices, pairs=64, groups=16, seed=0, noise=MCINV_NOISE_NORMAL, device=0,
                 rows_per_item=0, grab=0, use_torch_stream=False, schedule=0):
        stream = torch_stream() if use_torch_stream else None
        self.b = mcinv_batch_create(len(matrices), device=device, noise=noise, n_pairs=pairs, n_groups=groups,
                                    rows_per_item=rows_per_item, grab=grab, seed=seed, stream=stream,
                                    schedule=schedule)
        self.n = [m.n for m in matrices]
        self.P = pairs
        self.bdim = 0
        try:
            for j, m in enumerate(matrices):
                mcinv_batch_load_csr(self.b, j, m.n, m.nnz, m.row_ptr, m.col, m.val)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "b", None) is not None:
            mcinv_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def request(self, diag=True, block_dim=0, expected_samples=1):
        flags = (MCINV_REQ_DIAG if diag else 0) | (MCINV_REQ_BLOCK if block_dim > 0 else 0)
        self.bdim = block_dim
        mcinv_batch_set_requested(self.b, flags, block_dim, expected_samples)

    def set_block(self, m, rows, cols):
        mcinv_batch_set_block(self.b, m, rows, cols)

    def burn_in(self, sweeps):
        mcinv_batch_burn_in(self.b, sweeps)

    def burn_in_coupled(self, tol=5e-5, max_sweeps=10000):
        """Coupled burn-in of every matrix; returns (sweeps, largest difference)."""
        from ._binding import mcinv_batch_burn_in_coupled
        return mcinv_batch_burn_in_coupled(self.b, tol, max_sweeps)

    def sample(self, sweeps):
        mcinv_batch_sample(self.b, sweeps)

    def sample_until(self, rel_se, max_sweeps, check_every=10):
        return mcinv_batch_sample_until(self.b, rel_se, max_sweeps, check_every)

    def sample_until_each(self, rel_se, max_sweeps, check_every=10):
        """Each matrix stops at its own first check that meets rel_se."""
        from ._binding import mcinv_batch_sample_until_each
        return mcinv_batch_sample_until_each(self.b, rel_se, max_sweeps, check_every)

    def matrix_samples(self):
        """(samples per matrix, active flags)."""
        from ._binding import mcinv_batch_matrix_samples
        return mcinv_batch_matrix_samples(self.b, len(self.n))

    def diag(self, m):
        return mcinv_batch_read_estimates(self.b, m, MCINV_REQ_DIAG, self.n[m])

    def labels(self, m):
        """Surrogate training labels of matrix m: c_ii (C^-1)_ii and their
        standard errors (``mcinv_batch_read_labels``)."""
        return mcinv_batch_read_labels(self.b, m, self.n[m])

    def block(self, m):
        est, se = mcinv_batch_read_estimates(self.b, m, MCINV_REQ_BLOCK, self.bdim * self.bdim)
        return est.reshape(self.bdim, self.bdim), se.reshape(self.bdim, self.bdim)

    def state(self, m, which):
        return mcinv_batch_read_state(self.b, m, which, self.n[m], self.P)

    def autotune(self, sweeps_per_trial=2):
        return mcinv_batch_autotune(self.b, sweeps_per_trial)

    def info(self):
        return mcinv_batch_get_info(self.b)
