"""The paper's second example, the free Wilson-Dirac matrix (Sec. 3.2):
the generator against the printed rank and nonzero counts (Table 3), the
closed-form trace of the inverse against a dense inverse and against the
printed exact values (Tables 4 and 5), convergence of the Gauss-Seidel
iterations (Sec. 2.2), and the oracle's trace estimate against the exact
value within its Geyer standard error."""

import json
import os

import numpy as np
import pytest

import gen
import oracle
from oracle import theory

GOLD = os.path.join(os.path.dirname(__file__), "golden", "dirac_free_field.json")


def _cases():
    with open(GOLD) as f:
        return json.load(f)["cases"]


def test_gammas_anticommute_and_are_hermitian():
    g = gen.dirac_gammas()
    for i in range(4):
        assert np.allclose(g[i], g[i].conj().T)
        for j in range(4):
            assert np.allclose(g[i] @ g[j] + g[j] @ g[i], 2.0 * (i == j) * np.eye(4))


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"N{c['N']}")
def test_generator_matches_table3_and_exact_trace(case):
    m = gen.dirac(case["N"], case["K"])
    assert m.n == case["rank"] and m.nnz == case["nnz"]
    assert np.all(np.diff(m.row_ptr) == 14)
    tr = theory.dirac_free_trace(case["N"], case["K"])
    # printed to two decimals; the closed form agrees to 4e-8 relative
    assert abs(tr - case["exact_trace"]) <= 5e-8 * case["exact_trace"]


@pytest.mark.parametrize("N", [3, 4])
def test_closed_form_matches_dense_inverse(N):
    A = gen.to_dense(gen.dirac(N, 0.1))
    tr = np.trace(np.linalg.inv(A))
    assert abs(tr.imag) < 1e-9
    assert abs(tr.real - theory.dirac_free_trace(N, 0.1)) < 1e-9 * abs(tr.real)
    # translation invariance: every site has the same diagonal block trace
    d = np.diag(np.linalg.inv(A)).reshape(4, -1).sum(axis=0)
    assert np.allclose(d, d[0])


def test_gauss_seidel_iterations_converge():
    C = gen.to_dense(gen.dirac(4, 0.1))
    _, order, _ = oracle.greedy_color(gen.dirac(4, 0.1))
    Cp = C[np.ix_(order, order)]
    T, S, _ = theory.operators(Cp)
    assert theory.spectral_radius(T) < 0.9 and theory.spectral_radius(S) < 0.9


def test_oracle_trace_estimate_within_error():
    N, K = 4, 0.1
    m = gen.dirac(N, K)
    exact = theory.dirac_free_trace(N, K)
    run = oracle.Run(m, seed=77, pairs=8)
    run.burn_in(30)
    S = 1200
    run.request(S, diag=False, trace=True)
    run.sample(S)
    g = run.trace()
    est = g["mean"]
    assert abs(est.real - exact) <= 4.5 * g["se"]
    assert abs(est.imag) <= 4.5 * g["se"]
    assert g["se"] < 2e-3 * exact
