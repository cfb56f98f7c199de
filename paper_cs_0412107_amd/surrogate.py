"""Learned surrogate of diag(C^-1) with a sampler fallback.

Writing C = D (I + M), the series C^-1 = sum_k (-M)^k D^-1 gives
y_i = c_ii (C^-1)_ii = 1 + (M^2)_ii - (M^3)_ii + ...; a small network predicts
y_i from 32 local features of row i (``mcinv_features``), trained on the
sampler's estimates (eq 1/C, scaled to c_ii (C^-1)_ii by
``mcinv_batch_read_labels``) weighted by their standard errors.  A gate fitted
on validation matrices sends the rows whose validated error exceeds the
tolerance back to the sampler, whose stop check then covers only those rows.

Every step runs in ``libmcinv.so``; this module sequences the calls.
"""

from __future__ import annotations

import numpy as np

from . import _binding as B


def features(matrix, device=0):
    """[n][32] float32 features of a real matrix (CSR with row_ptr, col, val)."""
    return B.mcinv_features(device, matrix.n, matrix.nnz, matrix.row_ptr, matrix.col, matrix.val)


def init_params(seed):
    """W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)); hidden biases 0; output bias 1
    (y is close to 1).  Flat, in the library's parameter order."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (32, 128)) / np.sqrt(32)
    W2 = rng.uniform(-1, 1, (128, 128)) / np.sqrt(128)
    w3 = rng.uniform(-1, 1, 128) / np.sqrt(128)
    return np.concatenate([W1.ravel(), np.zeros(128), W2.ravel(), np.zeros(128), w3, [1.0]]).astype(np.float32)


class Network:
    """The 32 -> 128 -> 128 -> 1 network on the device (``mcinv_mlp``)."""

    def __init__(self, device=0, params=None, seed=1):
        self.h = B.mcinv_mlp_create(device)
        self.set_params(init_params(seed) if params is None else params)

    def close(self):
        if self.h:
            B.mcinv_mlp_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        B.mcinv_mlp_set_params(self.h, p)

    def params(self):
        return B.mcinv_mlp_get_params(self.h)

    def set_normalization(self, mean, inv_std):
        B.mcinv_mlp_set_normalization(self.h, mean, inv_std)

    def set_data(self, X, y, w, normalize=True):
        B.mcinv_mlp_set_data(self.h, X, y, w)
        if normalize:
            return B.mcinv_mlp_fit_normalization(self.h)
        return None

    def gradients(self, rows):
        return B.mcinv_mlp_gradients(self.h, rows)

    def train(self, steps, batch_rows=1024, lr=1e-3, seed=7):
        return B.mcinv_mlp_train(self.h, steps, batch_rows, lr, seed)

    def predict(self, X):
        return B.mcinv_mlp_predict(self.h, X)

    def estimate_matrix(self, matrix, gate):
        """(estimates of (C^-1)_ii, gate fallback flags) for a matrix, its
        features made and used on the device (``mcinv_mlp_estimate_matrix``)."""
        return B.mcinv_mlp_estimate_matrix(self.h, gate.h, matrix.n, matrix.nnz, matrix.row_ptr, matrix.col,
                                           matrix.val)


class Gate:
    """Per-bin validated error over two features (``mcinv_gate``)."""

    def __init__(self, X, pred, y, y_se, feature_a=1, feature_b=5, bins=8, min_rows=50, tol=0.01, ucb_z=0.0):
        self.bins = bins
        self.h = B.mcinv_gate_fit(X, pred, y, y_se, feature_a, feature_b, bins, min_rows, tol, ucb_z)

    def close(self):
        if self.h:
            B.mcinv_gate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fallback(self, X):
        return B.mcinv_gate_apply(self.h, X).astype(bool)

    def table(self):
        return B.mcinv_gate_read(self.h, self.bins)


def estimate_diag(matrix, net, gate, sampler_factory, rel_se=0.01, max_sweeps=20000, check_every=20,
                  burn_in=200):
    """diag(C^-1): the network's prediction where the gate accepts it, the
    sampler's estimate (stop check over the rejected rows only) elsewhere.

    ``sampler_factory(matrix)`` returns a ``Sampler`` for the matrix;
    ``burn_in`` is a sweep count or "coupled" (until the coupled paths agree
    to 5e-5).
    Returns (estimate, source) with source 0 = network, 1 = sampler, and a
    dict of counts and sweeps (with the sampler's standard errors of every row
    under "se" when any row fell back)."""
    est, fb = net.estimate_matrix(matrix, gate)
    fb = fb.astype(bool)
    info = {"rows": int(matrix.n), "fallback_rows": int(fb.sum()), "sweeps": 0}
    if fb.any():
        with sampler_factory(matrix) as s:
            if burn_in == "coupled":
                s.burn_in_coupled(5e-5, 10000)
            else:
                s.burn_in(burn_in)
            s.request(diag=True, trace=False)
            s.set_stop_rows(np.nonzero(fb)[0])
            done, achieved = s.sample_until(rel_se, max_sweeps, check_every)
            sd, sse = s.diag()
        est[fb] = np.asarray(sd).real[fb]
        info.update(sweeps=int(done), achieved=float(achieved), se=np.asarray(sse))
    return est, fb.astype(np.uint8), info
