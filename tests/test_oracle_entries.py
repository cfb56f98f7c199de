"""Pin of the oracle's entry moments (eq 1/C for i != j): the mean of
z_i conj(w_j) over samples estimates (C^-1)_ij.

A non-symmetric C has (C^-1)_ij != (C^-1)_ji, so the two index roles of the
accumulator are told apart: the estimates must sit within their errors of the
dense inverse, and, where the transposed entry differs from the exact one by
many errors, far away from the transposed value.  A complex non-hermitian C
also separates z_i conj(w_j) from the conjugated or unconjugated readings.
"""

import numpy as np
import pytest

import gen
import oracle


def _complex_variant(m, seed):
    """The same pattern with every stored off-diagonal entry turned by a random
    phase and the diagonal by a small one (still strictly row dominant)."""
    rng = np.random.default_rng(seed)
    A = gen.to_dense(m).astype(np.complex128)
    off = (A != 0) & ~np.eye(m.n, dtype=bool)
    A[off] *= np.exp(1j * rng.uniform(0, 2 * np.pi, size=off.sum()))
    A[np.diag_indices(m.n)] *= np.exp(1j * rng.uniform(-0.4, 0.4, size=m.n))
    return gen.from_dense(A)


def _run_entries(m, pairs, seed, samples):
    n = m.n
    ij = np.array([(i, j) for i in range(n) for j in range(n)], dtype=np.int64)
    r = oracle.Run(m, seed=seed, pairs=pairs, groups=32)
    r.burn_in(200)
    r.request(samples, diag=False, entries=ij, trace=False)
    r.sample(samples)
    est, se = r.entries()
    return ij, est, se


@pytest.mark.parametrize("cplx", [False, True])
def test_entries_against_dense_inverse_and_transpose(cplx):
    m = gen.random_dominant(24, 3, seed=4242, factor=1.3)
    if cplx:
        m = _complex_variant(m, 99)
    exact = np.linalg.inv(gen.to_dense(m))
    ij, est, se = _run_entries(m, pairs=128, seed=0x5EED, samples=3000)
    i, j = ij[:, 0], ij[:, 1]
    assert np.all(se > 0)

    # within their errors of the exact inverse (all 576 entries)
    z = np.abs(est - exact[i, j]) / se
    assert np.max(z) < 5.0
    # the complex SE is the modulus of the two parts' errors, so |z|^2 has mean
    # ~1 in both cases (t-distributed with 31 degrees of freedom: 1.07)
    assert 0.8 <= np.mean(z ** 2) <= 1.3
    zr = (est - exact[i, j]).real / se
    assert abs(zr.mean()) < 0.15
    if not cplx:
        assert np.max(np.abs(est.imag)) == 0.0

    # the transposed reading (i and j swapped) is far off where it differs
    far = np.abs(exact[i, j] - exact[j, i]) > 20 * se
    assert far.sum() >= 40
    zt = np.abs(est - exact[j, i]) / se
    assert np.min(zt[far]) >= 10.0

    if cplx:
        # neither conj(C^-1) nor the conjugate transpose matches
        for alt in (np.conj(exact[i, j]), np.conj(exact[j, i])):
            sep = np.abs(exact[i, j] - alt) > 20 * se
            assert sep.sum() >= 40
            assert np.min(np.abs(est - alt)[sep] / se[sep]) >= 10.0
