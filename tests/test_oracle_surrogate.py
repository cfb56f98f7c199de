"""Pins of the surrogate oracle (features, network, Adam, row draws, gate)
against what the mathematics fixes: brute-force loops over a dense matrix on
tiny inputs, the remainder bound of the Neumann series of C^-1, library
routines (torch's bfloat16 rounding and Adam), central finite differences of
the float64 network, and hand-computed gate bins.  The gate in the C library is
host code and is checked against the oracle here too."""

import numpy as np
import pytest

import gen
import oracle
from oracle import surrogate as S


def _tiny(seed, n=12):
    """Non-symmetric pattern, one isolated row, mixed signs, dominant diagonal."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < 0.3)
    np.fill_diagonal(A, 0)
    A[3, :] = 0
    A[:, 3] = 0
    d = 1.7 * np.maximum(np.abs(A).sum(axis=1), np.abs(A).sum(axis=0)) + 0.2
    d *= np.where(rng.random(n) < 0.25, -1.0, 1.0)
    A[np.diag_indices(n)] = d
    return A


def _brute_features(A):
    """Every feature from its definition with plain loops over the dense matrix."""
    n = A.shape[0]
    d = np.diag(A)
    m = lambda i, j: A[i, j] / d[i] if i != j else 0.0  # noqa: E731
    F = np.zeros((n, 32))
    nb = [[j for j in range(n) if j != i and (A[i, j] != 0 or A[j, i] != 0)] for i in range(n)]
    for i in range(n):
        r = [j for j in range(n) if j != i and A[i, j] != 0]
        c = [j for j in range(n) if j != i and A[j, i] != 0]
        F[i, 0] = np.log(abs(d[i]))
        F[i, 1] = sum(abs(A[i, j]) for j in r) / abs(d[i])
        F[i, 2] = sum(abs(A[j, i]) for j in c) / abs(d[i])
        F[i, 3] = len(r) / 8
        F[i, 4] = len(c) / 8
        F[i, 5] = sum(m(i, j) * m(j, i) for j in range(n))
        F[i, 6] = sum(m(i, j) * m(j, k) * m(k, i) for j in range(n) for k in range(n))
        F[i, 7] = sum(abs(m(i, j)) * abs(m(j, i)) for j in range(n))
        F[i, 8] = sum(m(i, j) ** 2 for j in range(n))
        F[i, 9] = sum(A[i, j] for j in r) / d[i]
        F[i, 10] = sum(A[j, i] for j in c) / d[i]
        F[i, 31] = 1.0
    for i in range(n):
        J = nb[i]
        F[i, 24] = len(J) / 8
        F[i, 25] = 1 + F[i, 5]
        F[i, 26] = 1 + F[i, 5] - F[i, 6]
        F[i, 27] = F[i, 1] ** 2
        F[i, 28] = F[i, 5] ** 2
        F[i, 29] = F[i, 5] * F[i, 1]
        F[i, 30] = sum(F[j, 1] ** 2 for j in J) / 8
        if not J:
            continue
        rv = np.array([F[j, 1] for j in J])
        lv = np.array([F[j, 0] for j in J])
        F[i, 11:15] = rv.mean(), rv.max(), rv.min(), rv.std()
        F[i, 15:18] = lv.mean() - F[i, 0], lv.max() - F[i, 0], lv.min() - F[i, 0]
        F[i, 18] = lv.std()
        q = np.array([F[j, 5] for j in J])
        F[i, 19:21] = q.mean(), q.max()
        cv = np.array([F[j, 2] for j in J])
        F[i, 21:23] = cv.mean(), cv.max()
        F[i, 23] = np.mean([F[j, 6] for j in J])
    return F


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_features_brute_force(seed):
    A = _tiny(seed)
    F = S.features(gen.from_dense(A))
    np.testing.assert_allclose(F, _brute_features(A), rtol=1e-12, atol=1e-13)
    assert np.all(F[3, 11:24] == 0) and F[3, 24] == 0  # isolated row: empty neighbourhood


def test_neumann_terms_match_the_inverse():
    """y_i = c_ii (C^-1)_ii = 1 + (M^2)_ii - (M^3)_ii + R_4 with |R_4| <= rho^4 / (1 - rho),
    rho = ||M||_inf: a wrong sign or index in features 5, 6 or 26 breaks the bound."""
    m = gen.random_dominant(150, 4, seed=77, factor=4.0)
    A = gen.to_dense(m).real
    y = np.diag(A) * np.diag(np.linalg.inv(A))
    F = S.features(m)
    rho = np.max(np.abs(A - np.diag(np.diag(A))).sum(axis=1) / np.abs(np.diag(A)))
    assert rho < 0.3
    bound = rho ** 4 / (1 - rho)
    assert np.max(np.abs(y - F[:, 26])) <= bound
    assert np.max(np.abs(y - F[:, 25])) > np.max(np.abs(y - F[:, 26]))  # the cubic term helps
    assert np.allclose(F[:, 25], 1 + F[:, 5]) and np.all(F[:, 31] == 1)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.float32(1) + np.float32(2.0 ** -8) * np.arange(0, 8),  # ties to even
                        [0.0, -0.0, 1.0, -3.5, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), ref)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(5)
    p = S.init_params(6)
    for k in ("b1", "b2"):
        p[k] = rng.uniform(-0.3, 0.3, p[k].shape)
    X = rng.standard_normal((40, S.NF))
    y = 1 + 0.1 * rng.standard_normal(40)
    w = rng.uniform(0.5, 2.0, 40)
    g = S.mlp_grads(p, X, y, w, bf16_ops=False, denom=40.0)
    h = 1e-6
    for k in S.ORDER:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = S.mlp_loss(p, X, y, w, bf16_ops=False, denom=40.0)
            flat[idx] = old - h
            lm = S.mlp_loss(p, X, y, w, bf16_ops=False, denom=40.0)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[k].reshape(-1)[idx] - fd) <= 1e-7 + 1e-5 * abs(fd), (k, idx)


def test_bf16_network_within_rounding_bound():
    """bf16 operands perturb each product by O(2^-8) relative: the gradients of the
    two networks agree to a few percent, and not to 1e-6 (the rounding is really applied)."""
    rng = np.random.default_rng(7)
    p = S.init_params(8)
    X = rng.standard_normal((256, S.NF))
    y = 1 + 0.1 * rng.standard_normal(256)
    w = np.ones(256)
    g64 = S.mlp_grads(p, X, y, w, bf16_ops=False)
    g16 = S.mlp_grads(p, X, y, w, bf16_ops=True)
    for k in S.ORDER:
        rel = np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k])
        assert rel < 0.05, k
    assert np.linalg.norm(g16["W1"] - g64["W1"]) > 1e-6 * np.linalg.norm(g64["W1"])


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    p = {k: rng.standard_normal(v.shape) for k, v in S.init_params(1).items()}
    tp = {k: torch.tensor(v.copy(), dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    st = {}
    for _ in range(4):
        g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
        p = S.adam_step(p, g, st, 1e-2)
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
    for k in p:
        np.testing.assert_allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14)


def test_flatten_order():
    p = S.init_params(2)
    v = S.flatten(p)
    assert v.size == S.N_PARAMS == 20865
    assert v[0] == p["W1"][0, 0] and v[1] == p["W1"][0, 1] and v[128] == p["W1"][1, 0]
    assert v[-1] == p["b3"][0] and v[-2] == p["w3"][-1]
    q = S.unflatten(v)
    assert all(np.array_equal(q[k], p[k]) for k in S.ORDER)


def test_batch_rows_power_of_two():
    """For N = 2^k the row is the top k bits of the first Philox output word."""
    seed = 0x1234_5678_9ABC
    rows = S.batch_rows(seed, 3, 1 << 10, 64)
    for r in range(64):
        o = oracle.philox4x32_10((r, 3, 0x5EED, 0xA11CE), (seed & 0xFFFFFFFF, seed >> 32))
        assert rows[r] == int(o[0]) >> 22
    big = S.batch_rows(seed, 1, 1000, 4000)
    assert big.min() >= 0 and big.max() < 1000 and len(np.unique(big)) > 900


def test_gate_hand_example():
    X = np.zeros((8, 32), dtype=np.float32)
    X[:, 0] = np.arange(8)
    X[:, 1] = [0, 1, 0, 1, 0, 1, 0, 1]
    y = np.ones(8)
    pred = np.array([1.0, 1.0, 1.0, 1.0, 1.1, 1.1, 1.0, 1.0])
    se = np.zeros(8)
    g = S.gate_fit(X, pred, y, se, 0, 1, 2, 1, 0.05)
    assert g["edges_a"].tolist() == [4.0] and g["edges_b"].tolist() == [1.0]
    # bins: (a, b) = (row >= 4, odd row)
    assert g["count"].tolist() == [2, 2, 2, 2]
    np.testing.assert_allclose(g["err"], [0, 0, np.sqrt(0.01 / 2), np.sqrt(0.01 / 2)], atol=1e-15)
    assert g["fallback"].tolist() == [False, False, True, True]
    Xq = X[[0, 5, 6]].copy()
    assert S.gate_apply(g, Xq).tolist() == [0, 1, 1]
    Xq[0, 1] = np.nan
    assert S.gate_apply(g, Xq)[0] == 1
    # label noise explains part of the spread
    g2 = S.gate_fit(X, pred, y, np.full(8, 0.05), 0, 1, 2, 1, 0.05)
    np.testing.assert_allclose(g2["err"][2], np.sqrt((0.01 - 2 * 0.0025) / 2), rtol=1e-12)
    g3 = S.gate_fit(X, pred, y, np.full(8, 0.08), 0, 1, 2, 1, 0.05)
    assert g3["err"][2] == 0.0  # noise larger than the spread


def test_chi2_lower_quantile_matches_scipy_and_covers():
    """The gate's confidence bound: Wilson-Hilferty against scipy's chi-square
    quantiles, and the bound covers the true RMS error ~95% of the time."""
    from scipy import stats
    z = 1.645
    for k in (20, 50, 200, 2000, 100000):
        exact = stats.chi2.ppf(stats.norm.cdf(-z), k)
        assert abs(S.chi2_lower_quantile(k, z) - exact) <= 0.01 * exact, k
    for k in (5, 10):
        exact = stats.chi2.ppf(stats.norm.cdf(-z), k)
        assert abs(S.chi2_lower_quantile(k, z) - exact) <= 0.05 * exact, k
    rng = np.random.default_rng(3)
    sigma, k, reps = 0.004, 30, 4000
    r = rng.normal(0.0, sigma, (reps, k))
    ucb = np.sqrt((r ** 2).sum(axis=1) / S.chi2_lower_quantile(k, z))
    cover = np.mean(ucb >= sigma)
    assert 0.93 < cover < 0.97, cover
    # in the gate: a small bin needs a smaller observed error than a large one.
    # Features 0 and 1 are ranks 0..209 split at 105; swapping rows 100-104 with
    # 105-109 in feature 1 leaves 100 rows in bins (0,0) and (1,1), 5 in (0,1), (1,0)
    X = np.zeros((210, 32), dtype=np.float32)
    X[:, 0] = np.arange(210)
    b = np.arange(210)
    b[100:105], b[105:110] = np.arange(105, 110), np.arange(100, 105)
    X[:, 1] = b
    y = np.ones(210)
    pred = 1 + np.where(np.arange(210) % 2 == 0, 0.008, -0.008)
    g0 = S.gate_fit(X, pred, y, np.zeros(210), 0, 1, 2, 1, 0.01)
    g = S.gate_fit(X, pred, y, np.zeros(210), 0, 1, 2, 1, 0.01, ucb_z=z)
    assert g0["count"].tolist() == [100, 5, 5, 100]
    np.testing.assert_allclose(g0["err"], 0.008, rtol=1e-12)
    # 100 rows: 0.008 sqrt(100 / q(100)) ~ 0.0091 <= 0.01; 5 rows: ~0.0168 > 0.01
    assert g["err"][0] < 0.01 < g["err"][1] and g["err"][3] < 0.01 < g["err"][2]
    assert g["fallback"].tolist() == [False, True, True, False]
    assert not g0["fallback"].any()
    # rows beyond the validated range of either binning feature fall back even
    # though their (open-ended) outer bin is trusted; the range's own ends do not
    Xq = np.zeros((6, 32), dtype=np.float32)
    Xq[:, 0] = [0, 209, -1, 210, 50, 50]
    Xq[:, 1] = [0, 209, 0, 0, -0.5, 1000]
    assert S.gate_apply(g0, Xq).tolist() == [0, 0, 1, 1, 1, 1]


def test_gate_library_matches_oracle():
    mc = pytest.importorskip("paper_cs_0412107_amd")
    try:
        mc.lib()
    except ImportError:
        pytest.skip("library not built")
    rng = np.random.default_rng(11)
    N = 5000
    X = rng.standard_normal((N, 32)).astype(np.float32)
    X[:, 5] = np.round(X[:, 5], 1)  # ties at the edges
    y = 1 + 0.2 * rng.random(N)
    pred = y * (1 + 0.01 * rng.standard_normal(N) * (1 + np.abs(X[:, 1])))
    se = 0.003 * y
    for bins, min_rows, tol, z in ((8, 20, 0.012, 0.0), (1, 1, 0.02, 0.0), (16, 30, 0.01, 0.0),
                                   (8, 5, 0.012, 1.645), (16, 2, 0.01, 2.33)):
        ref = S.gate_fit(X, pred, y, se, 1, 5, bins, min_rows, tol, ucb_z=z)
        h = mc.mcinv_gate_fit(X, pred, y, se, 1, 5, bins, min_rows, tol, ucb_z=z)
        try:
            got = mc.mcinv_gate_read(h, bins)
            assert np.array_equal(got["edges_a"], ref["edges_a"])
            assert np.array_equal(got["edges_b"], ref["edges_b"])
            assert np.array_equal(got["count"], ref["count"])
            np.testing.assert_allclose(got["err"], ref["err"], rtol=1e-12)
            assert np.array_equal(got["fallback"], ref["fallback"])
            assert got["range_a"] == ref["range_a"] and got["range_b"] == ref["range_b"]
            Xq = rng.standard_normal((777, 32)).astype(np.float32) * 1.5
            Xq[::50, 1] = np.nan
            Xq[3::50, 5] = 1e6   # beyond the validated range
            out = mc.mcinv_gate_apply(h, Xq)
            assert np.array_equal(out, S.gate_apply(ref, Xq))
            assert out[3::50].all() and out[::50].all()
        finally:
            mc.mcinv_gate_destroy(h)
    with pytest.raises(mc.McinvError):
        mc.mcinv_gate_fit(X, pred, y, se, 1, 40, 8, 1, 0.01)


def test_label_weights_library_matches_oracle():
    mc = pytest.importorskip("paper_cs_0412107_amd")
    try:
        mc.lib()
    except ImportError:
        pytest.skip("library not built")
    se = np.random.default_rng(2).uniform(0.0, 0.03, 1000)
    w = S.label_weights(se, 1e-6)
    assert abs(w.mean() - 1) < 1e-12 and np.all(np.diff(w[np.argsort(se)]) <= 0)
    np.testing.assert_allclose(mc.mcinv_mlp_label_weights(se, 1e-6), w, rtol=1e-6)


def test_fit_normalization_standardises():
    """After (x - mean) * inv_std every non-constant column has mean 0 and
    population variance 1; a constant column gets inv_std 1 (so it maps to 0)."""
    rng = np.random.default_rng(13)
    X = (rng.standard_normal((4000, 32)) * rng.uniform(0.01, 50, 32) + rng.uniform(-5, 5, 32)).astype(np.float32)
    X[:, 31] = 1.0
    mean, inv = S.fit_normalization(X)
    Z = S.normalize(X, mean, inv)
    assert np.allclose(Z[:, :31].mean(axis=0), 0, atol=1e-5)
    assert np.allclose(Z[:, :31].var(axis=0), 1, rtol=1e-5)
    assert inv[31] == 1.0 and np.all(Z[:, 31] == 0)
