"""Pins of the oracle sweep and estimators against what the paper and the
mathematics fix: the exact finite-sweep expectation of the demonstration
(Sec. 2.1), its recursion, exact special cases (diagonal, triangular,
hermitian C), the coupling identity of Sec. 2.3 (eq 12), the convergence
condition of Sec. 2.2, and the dense LU inverse."""

import numpy as np
import pytest
from scipy.linalg import solve_triangular

import gen
import oracle
from oracle import theory


def _dense_random(n, seed, cplx=False, factor=1.6, density=0.6):
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < density)
    if cplx:
        A = A + 1j * rng.uniform(-1, 1, (n, n)) * (A != 0)
    np.fill_diagonal(A, 0)
    d = factor * np.abs(A).sum(axis=1) + 0.1
    if cplx:
        d = d * np.exp(1j * rng.uniform(-0.6, 0.6, n))
    A[np.diag_indices(n)] = d
    return A


# --- P8: the demonstration's operators ----------------------------------------
@pytest.mark.parametrize("cplx", [False, True])
def test_recursion_and_series_limit(cplx):
    C = _dense_random(7, 1, cplx)
    T, S, Y = theory.operators(C)
    Ci = np.linalg.inv(C)
    assert np.allclose(Ci, Y + T @ Ci @ S, atol=1e-13, rtol=0)
    assert np.allclose(theory.expected_zw(C, 200), Ci, atol=1e-12, rtol=0)
    assert theory.spectral_radius(T) < 1 and theory.spectral_radius(S) < 1


# --- P2: exact expectation after k sweeps from z = w = 0 ------------------------
@pytest.mark.parametrize("cplx,perm", [(False, False), (True, False), (True, True)])
def test_finite_sweep_expectation(cplx, perm):
    n, P = 6, 60_000
    C = _dense_random(n, 2 + cplx, cplx, factor=1.1)
    m = gen.from_dense(C)
    order = np.random.default_rng(9).permutation(n) if perm else np.arange(n)
    Cp = C[np.ix_(order, order)]  # the matrix the sweep sees
    run = oracle.Run(m, seed=123, pairs=P, order=order)
    worst = 0.0
    for k in (1, 2, 3):
        run.burn_in(1)
        prod = run.z[:, None, :] * np.conj(run.w[None, :, :])  # [i, j, p]
        mean = prod.mean(axis=2)
        se = np.sqrt(prod.real.var(axis=2) / P + prod.imag.var(axis=2) / P)
        exp_p = theory.expected_zw(Cp, k)
        inv = np.argsort(order)
        expected = exp_p[np.ix_(inv, inv)]
        zs = np.abs(mean - expected) / np.maximum(se, 1e-300)
        worst = max(worst, zs.max())
        # a wrong sweep (old values instead of new, transposed w operand) is
        # off by many standard errors at k = 2, 3
    assert worst < 5.0


def test_finite_sweep_expectation_detects_jacobi():
    """The same statistic separates the Gauss-Seidel expectation from the one a
    Jacobi-style sweep (all neighbours from the previous sweep) would have."""
    n, P = 6, 60_000
    C = _dense_random(n, 5, False, factor=1.1)
    run = oracle.Run(gen.from_dense(C), seed=5, pairs=P, order=np.arange(n))
    run.burn_in(2)
    prod = run.z[:, None, :] * np.conj(run.w[None, :, :])
    mean = prod.mean(axis=2).real
    se = np.sqrt(prod.real.var(axis=2) / P)
    D = np.diag(np.diag(C))
    Dinv = np.linalg.inv(D)
    J = -Dinv @ (C - D)
    jac = Dinv + J @ Dinv @ np.conj(J).T  # two Jacobi steps from zero
    assert np.max(np.abs(mean - jac) / se) > 8.0
    assert np.max(np.abs(mean - theory.expected_zw(C, 2).real) / se) < 5.0


# --- P3: diagonal C -------------------------------------------------------------
@pytest.mark.parametrize("cplx", [False, True])
def test_diagonal_exact(cplx):
    d = np.array([2.0, -3.0, 0.5, 7.25]) if not cplx else np.array([2.0, -3.0, 0.5 + 1j, -1 - 2j])
    m = gen.diag_matrix(d)
    run = oracle.Run(m, seed=77, pairs=8, order=np.arange(4), noise_kind=oracle.NOISE_RADEMACHER)
    for _ in range(3):
        run.burn_in(1)
        prod = run.z * np.conj(run.w)
        assert np.allclose(prod, (1.0 / d)[:, None], rtol=1e-15, atol=0)
    run = oracle.Run(m, seed=77, pairs=8, order=np.arange(4))
    run.burn_in(2)
    phi = oracle.noise(77, 0, np.arange(4)[:, None], 1, np.arange(8)[None, :])
    assert np.allclose(run.z * np.conj(run.w), phi ** 2 / d[:, None], rtol=1e-14, atol=0)


# --- P4: triangular C forgets its initial value after one sweep -----------------
@pytest.mark.parametrize("lower", [True, False])
def test_triangular_memoryless(lower):
    C = _dense_random(6, 8, True)
    C = np.tril(C) if lower else np.triu(C)
    m = gen.from_dense(C)
    runs = []
    for init in (0.0, 1.0):
        r = oracle.Run(m, seed=3, pairs=4, order=np.arange(6))
        r.z[:] = init * (np.arange(6)[:, None] + 1.0)
        r.w[:] = init * (np.arange(6)[:, None] - 2.0j)
        r.burn_in(1)
        runs.append(r)
    if lower:  # U = 0: z uses only new values; w = eq (5) on C^dagger (upper) does not
        assert np.array_equal(runs[0].z, runs[1].z)
        assert not np.array_equal(runs[0].w, runs[1].w)
    else:
        assert np.array_equal(runs[0].w, runs[1].w)
        assert not np.array_equal(runs[0].z, runs[1].z)


# --- P5: hermitian C reduces to the single-draw sampler (z = w) ------------------
def test_hermitian_z_equals_w():
    A = _dense_random(8, 11, True)
    H = (A + np.conj(A.T)) / 2
    H[np.diag_indices(8)] = 3.0 * np.abs(H).sum(axis=1)
    r = oracle.Run(gen.from_dense(H), seed=5, pairs=12)
    r.burn_in(7)
    assert np.array_equal(r.z, r.w)


# --- P6: coupling (Sec. 2.3, eq 12) ----------------------------------------------
def test_coupling_difference_is_gauss_seidel():
    n = 7
    C = _dense_random(n, 12, True, factor=1.05)
    m = gen.from_dense(C)
    r1 = oracle.Run(m, seed=21, pairs=4, order=np.arange(n))
    r2 = oracle.Run(m, seed=21, pairs=4, order=np.arange(n))
    z0 = np.arange(n, dtype=np.complex128)  # Algorithm 1, step 1: z* = i
    r2.z[:] = z0[:, None]
    r2.w[:] = z0[:, None]
    L, D, U = theory.split(C)
    x = z0.copy()
    y = z0.copy()
    for _ in range(25):
        r1.burn_in(1)
        r2.burn_in(1)
        x = solve_triangular(D + L, -U @ x, lower=True)                     # GS on C x = 0
        y = solve_triangular(np.conj(D + U).T, -np.conj(L).T @ y, lower=True)  # on C^dagger y = 0
        for p in range(4):
            assert np.allclose(r2.z[:, p] - r1.z[:, p], x, rtol=0, atol=1e-12 * max(1, abs(z0).max()))
            assert np.allclose(r2.w[:, p] - r1.w[:, p], y, rtol=0, atol=1e-12 * max(1, abs(z0).max()))


def test_coupling_contraction_rate_is_spectral_radius():
    rng = np.random.default_rng(13)
    C = -rng.uniform(0.2, 1.0, (9, 9))  # same-sign couplings: sp(T) near 1
    np.fill_diagonal(C, 0)
    np.fill_diagonal(C, 1.05 * np.abs(C).sum(axis=1))
    m = gen.from_dense(C)
    T, S, _ = theory.operators(C)
    r1 = oracle.Run(m, seed=1, pairs=1, order=np.arange(9))
    r2 = oracle.Run(m, seed=1, pairs=1, order=np.arange(9))
    r2.z[:] = np.arange(9)[:, None] + 1.0
    r2.burn_in(40)
    r1.burn_in(40)
    d40 = np.abs(r2.z - r1.z).max()
    r1.burn_in(60)
    r2.burn_in(60)
    d100 = np.abs(r2.z - r1.z).max()
    rate = (d100 / d40) ** (1 / 60)
    assert abs(rate - theory.spectral_radius(T)) < 0.02


def test_coupled_burn_in_length_is_gauss_seidel_closed_form():
    """Algorithm 1 steps 1-5 run literally (two noisy paths) stop at the first k
    with ||G^k x*|| < tol for the dense Gauss-Seidel matrices G of C and C^dagger
    (eq 12), x*_i = i: an off-by-one in the count, a wrong start or a w path
    swept on C instead of C^dagger changes N or the differences."""
    n = 12
    C = _dense_random(n, 31, True, factor=1.15)
    m = gen.from_dense(C)
    order = np.arange(n)
    N, diffs = oracle.coupled_burn_in(m, seed=8, tol=1e-6, max_sweeps=400, order=order)
    L, D, U = theory.split(C)
    x = np.arange(1, n + 1, dtype=np.complex128)
    y = x.copy()
    k_ref = None
    for k in range(1, 401):
        x = solve_triangular(D + L, -U @ x, lower=True)
        y = solve_triangular(np.conj(D + U).T, -np.conj(L).T @ y, lower=True)
        dz, dw = np.abs(x).max(), np.abs(y).max()
        if k <= len(diffs):
            assert abs(diffs[k - 1][0] - dz) <= 1e-10 * n and abs(diffs[k - 1][1] - dw) <= 1e-10 * n
        if dz < 1e-6 and dw < 1e-6:
            k_ref = k
            break
    assert k_ref is not None and N == k_ref and N > 5


# --- P9: convergence condition (Sec. 2.2) -----------------------------------------
@pytest.mark.parametrize("maker", [
    lambda: gen.random_dominant(200, seed=1000),
    lambda: gen.pedigree(400, seed=7),
    lambda: gen.lattice(4, seed=2),
])
def test_generated_matrices_converge(maker):
    C = gen.to_dense(maker())
    T, S, _ = theory.operators(C)
    assert theory.spectral_radius(T) < 1 and theory.spectral_radius(S) < 1


def test_divergence_detected():
    C = np.array([[1.0, 2.5, 0.0], [2.0, 1.0, 1.5], [0.0, 3.0, 1.0]])
    T, _, _ = theory.operators(C)
    assert theory.spectral_radius(T) > 1
    r = oracle.Run(gen.from_dense(C), seed=1, pairs=2, order=np.arange(3))
    with pytest.raises(oracle.OracleError, match="diverged"):
        r.burn_in(2000)


def test_zero_diagonal_rejected():
    C = np.array([[1.0, 0.5], [0.5, 0.0]])
    r = oracle.Run(gen.from_dense(C), seed=1, pairs=1, order=np.arange(2))
    with pytest.raises(oracle.OracleError, match="diagonal"):
        r.burn_in(1)


# --- P7: lattice closed form ------------------------------------------------------
def test_lattice_closed_form_matches_dense_inverse():
    m = gen.lattice(4, k=0.1, seed=31, constant_phase=True)
    pr = m.params
    d, tr = theory.lattice_constant_phase_inverse_diag(4, pr["k"], pr["a"], pr["b"],
                                                       pr["theta"], pr["theta_p"])
    Ci = np.linalg.inv(gen.to_dense(m))
    assert np.allclose(np.diag(Ci), d, atol=1e-13)
    assert abs(np.trace(Ci) - tr) < 1e-11
    assert abs(d.imag) > 1e-4  # genuinely complex


def test_lattice_estimates_within_error():
    m = gen.lattice(4, k=0.1, seed=31, constant_phase=True)
    pr = m.params
    d, tr = theory.lattice_constant_phase_inverse_diag(4, pr["k"], pr["a"], pr["b"],
                                                       pr["theta"], pr["theta_p"])
    r = oracle.Run(m, seed=0x412109, pairs=64, groups=16)
    r.burn_in(30)
    r.request(200, diag=True, trace=True)
    r.sample(200)
    est, se = r.diag()
    z = np.abs(est - d) / se
    assert np.mean(z) < 1.6 and np.max(z) < 5.5
    t = r.trace()
    assert abs(t["mean"] - tr) < 5 * t["se"]


# --- eq tr with a general Q (Algorithm 1, step 8) ---------------------------------
def test_qtrace_estimates_tr_QCinv_not_its_conjugate():
    """E[w^dagger Q z] = tr(Q C^-1).  With complex non-hermitian C and Q the
    conjugate reading tr(Q C^-dagger) is many standard errors away."""
    import scipy.sparse as sp
    n = 10
    C = _dense_random(n, 41, True, factor=1.3)
    rng = np.random.default_rng(42)
    Qd = (rng.uniform(-1, 1, (n, n)) + 1j * rng.uniform(-1, 1, (n, n))) * (rng.random((n, n)) < 0.3)
    Qd += 3j * np.eye(n)
    Ci = np.linalg.inv(C)
    exact = np.trace(Qd @ Ci)
    wrong = np.trace(Qd @ Ci.conj().T)
    run = oracle.Run(gen.from_dense(C), seed=3, pairs=64)
    run.burn_in(30)
    run.request(600, diag=False, trace=True)
    run.set_trace_matrix(sp.csr_matrix(Qd))
    run.sample(600)
    g = run.qtrace()
    assert abs(g["mean"] - exact) <= 4.5 * g["se"]
    assert abs(g["mean"] - wrong) >= 10 * g["se"]
    # Q = I reproduces the plain trace series of eq tr
    run2 = oracle.Run(gen.from_dense(C), seed=3, pairs=64)
    run2.burn_in(30)
    run2.request(50, diag=False, trace=True)
    run2.set_trace_matrix(sp.identity(n, format="csr"))
    run2.sample(50)
    assert np.allclose(np.array(run2.qseries), run2.series[:50], rtol=1e-13, atol=0)
