"""Helpers shared by the GPU tests (comparison of library output with the
oracle on the same seeded inputs)."""

import numpy as np

import gen
import oracle

STATE_DTYPE = {"f32": np.float32, "f64": np.float64, "c64": np.complex64, "c128": np.complex128}
TOL = {"f32": 1e-5, "c64": 1e-5, "f64": 1e-12, "c128": 1e-12}


def oracle_matrix(m, dtype):
    """The matrix the oracle must see for a given sweep precision: 32-bit
    sweeps work on the 32-bit rounded values."""
    if dtype in ("f32", "c64"):
        return gen.round_values(m, np.float32 if not m.is_complex else np.complex64)
    return m


def rel_err(a, b):
    """Normwise relative error max|a-b| / max|b|."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def make_oracle(m, dtype, seed, pairs, groups=1, pair_ids=None, noise=oracle.NOISE_NORMAL, stream=0):
    return oracle.Run(oracle_matrix(m, dtype), seed=seed, pairs=pairs, groups=groups, pair_ids=pair_ids,
                      noise_kind=noise, stream=stream)


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
