"""Pins of the oracle's noise: Philox4x32-10 known answers and the law of the
normal / Z2 noise (eqs 5a, 5b: zero mean, identity covariance, independent)."""

import json
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLD, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x, 16) for x in v["out"]]
        assert list(oracle.philox4x32_10(ctr, key)) == out


def _draws(kind, rows=25_000, seed=0x412107):
    r = np.repeat(np.arange(rows), 4)
    p = np.tile(np.arange(4), rows)
    return oracle.noise(seed, 0, r, 3, p, kind)


def test_normal_noise_moments_and_ks():
    x = _draws(oracle.NOISE_NORMAL)
    n = x.size
    assert abs(x.mean()) < 4.0 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 4.0 * np.sqrt(2.0 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # the four outputs of one Philox block are uncorrelated (eq 5b, off-diagonal)
    q = x.reshape(-1, 4)
    c = np.corrcoef(q.T)
    assert np.max(np.abs(c - np.eye(4))) < 4.0 / np.sqrt(q.shape[0])


def test_rademacher_noise():
    x = _draws(oracle.NOISE_RADEMACHER, rows=10_000)
    assert set(np.unique(x)) == {-1.0, 1.0}
    assert abs(x.mean()) < 4.0 / np.sqrt(x.size)


def test_noise_counter_layout():
    """Pair p takes output p mod 4 of the block with counter (row, sweep, p div 4,
    stream); different streams, sweeps and rows give different blocks."""
    blk = np.zeros(4)
    lib = oracle.lib()
    buf = np.zeros(4, dtype=np.float64)
    lib.ora_noise_block(7, 0, 11, 5, 2, oracle.NOISE_NORMAL, buf.ctypes.data)
    blk[:] = buf
    for p in range(8, 12):
        assert oracle.noise(7, 0, 11, 5, p) == blk[p % 4]
    assert oracle.noise(7, 1, 11, 5, 8) != blk[0]
    assert oracle.noise(7, 0, 11, 6, 8) != blk[0]
    assert oracle.noise(7, 0, 12, 5, 8) != blk[0]
    assert oracle.noise(8, 0, 11, 5, 8) != blk[0]


@pytest.mark.parametrize("x", [0, 1, 511, 512, 0xFFFFFFFF, 0x80000000])
def test_uniform_open_interval(x):
    u = oracle.lib().ora_uniform
    import ctypes
    u.argtypes = [ctypes.c_uint32]
    u.restype = ctypes.c_double
    v = u(x)
    assert 0.0 < v < 1.0
    assert v == ((x >> 9) + 0.5) / 2 ** 23
    assert np.float32(v) == v  # exactly representable in binary32 too
