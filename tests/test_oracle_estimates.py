"""Statistical pins of the oracle's estimators: the tiny real non-symmetric
workload against its dense LU inverse (eq 1/C), the 1/sqrt(samples) error
law, and the calibration of the reported standard errors against replicated
runs (the paper's own check, Sec. 3.1: one hundred replicates with different
seeds)."""

import json
import os

import numpy as np
import pytest

import gen
import oracle
from oracle import cluster_estimate, geyer_ips

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_tables_se_relation():
    """Tables 2, 4, 5 obey SE = sqrt(Var / N_eff) -- the relation the Geyer
    finalisation implements -- and stop below the stated relative tolerance."""
    with open(os.path.join(GOLD, "paper_tables.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        assert abs(np.sqrt(r["var"] / r["n_eff"]) - r["se"]) <= 0.0015 * r["se"] + 5e-4
        assert r["se"] / abs(r["estimate"]) < r["tol"]


def test_geyer_ar1_closed_form():
    """AR(1) x_t = rho x_{t-1} + e_t: integrated autocorrelation time
    (1 + rho) / (1 - rho), stationary variance 1 / (1 - rho^2)."""
    rng = np.random.default_rng(0)
    rho, S = 0.6, 400_000
    e = rng.standard_normal(S)
    x = np.empty(S)
    x[0] = e[0] / np.sqrt(1 - rho ** 2)
    for t in range(1, S):
        x[t] = rho * x[t - 1] + e[t]
    g = geyer_ips(x)
    tau = (1 + rho) / (1 - rho)
    assert abs(g["n_eff"] / (S / tau) - 1) < 0.05
    assert abs(g["var"] * (1 - rho ** 2) - 1) < 0.02
    assert abs(g["se"] / np.sqrt(tau / (1 - rho ** 2) / S) - 1) < 0.05
    # independent samples: N_eff ~ S
    gi = geyer_ips(e)
    assert abs(gi["n_eff"] / S - 1) < 0.05


def test_cluster_estimate_equal_weights_closed_form():
    rng = np.random.default_rng(1)
    sums = rng.standard_normal((40, 3)) * 10 + 5
    counts = np.full(40, 10.0)
    est, se = cluster_estimate(sums, counts)
    means = sums / 10.0
    assert np.allclose(est, means.mean(axis=0), rtol=1e-14)
    assert np.allclose(se, means.std(axis=0, ddof=1) / np.sqrt(40), rtol=1e-12)


@pytest.fixture(scope="module")
def tiny_run():
    """The tiny workload: n=200 real non-symmetric, one chain pair, 500 burn-in
    sweeps and 20000 samples, the whole 200 x 200 inverse requested."""
    w = gen.WORKLOADS["tiny"]
    m = gen.random_dominant(w["n"], w["offdiag"], seed=w["seed"])
    r = oracle.Run(m, seed=w["noise_seed"], pairs=1, groups=1)
    r.burn_in(w["burn_in"])
    allrows = np.arange(m.n)
    r.request(w["samples"], diag=True, block_rows=allrows, block_cols=allrows, trace=True)
    exact = np.linalg.inv(gen.to_dense(m))
    rms = {}
    done = 0
    for S in (1250, 5000, 20000):
        r.sample(S - done)
        done = S
        est = r.block_acc.sum(axis=(0, 1)) / r.counts.sum()
        rms[S] = np.sqrt(np.mean(np.abs(est - exact) ** 2))
    return m, r, exact, rms


def test_tiny_inverse_zscores(tiny_run):
    m, r, exact, _ = tiny_run
    est, se = r.block()
    assert np.max(np.abs(est.imag)) == 0.0
    z = (est.real - exact) / se
    assert abs(z.mean()) < 0.05
    assert 0.9 <= z.std() <= 1.1
    assert np.mean(np.abs(z) > 4) <= 1e-3
    assert np.max(np.abs(z)) <= 6.0
    d, dse = r.diag()
    assert np.allclose(d.real, np.diag(est.real), rtol=1e-12)
    t = r.trace()
    assert abs(t["mean"].real - np.trace(exact)) < 5 * t["se"]


def test_tiny_error_law(tiny_run):
    _, _, _, rms = tiny_run
    S = np.array(sorted(rms))
    e = np.array([rms[s] for s in S])
    slope = np.polyfit(np.log(S), np.log(e), 1)[0]
    assert -0.6 <= slope <= -0.4


def test_se_calibration_replicates():
    """Empirical spread of 120 seed replicates vs the mean reported SE, for
    the diagonal (batch means) and the trace (Geyer)."""
    m = gen.random_dominant(16, 3, seed=77, factor=1.3)
    exact = np.linalg.inv(gen.to_dense(m))
    diag_est, diag_se, tr_est, tr_se = [], [], [], []
    for rep in range(120):
        r = oracle.Run(m, seed=1000 + rep, pairs=1, groups=1)
        r.burn_in(50)
        r.request(3000, diag=True, trace=True)
        r.sample(3000)
        d, s = r.diag()
        diag_est.append(d.real)
        diag_se.append(s)
        t = r.trace()
        tr_est.append(t["mean"].real)
        tr_se.append(t["se"])
    diag_est = np.array(diag_est)
    ratio = diag_est.std(axis=0, ddof=1) / np.mean(diag_se, axis=0)
    assert 0.85 <= ratio.mean() <= 1.15
    tr_ratio = np.std(tr_est, ddof=1) / np.mean(tr_se)
    assert 0.85 <= tr_ratio <= 1.15
    z = (diag_est.mean(axis=0) - np.diag(exact)) / (diag_est.std(axis=0, ddof=1) / np.sqrt(120))
    assert np.max(np.abs(z)) < 4.5
