"""Dense closed forms from the paper's demonstration (test infrastructure only).

Sec. 2.1 writes the sweep in matrix form with C = L + D + U (strict lower,
diagonal, strict upper) and derives, for zero initial values,

    E[z^(k) w^(k)dagger] = sum_{m=0}^{k-1} T^m Y S^m,
    T = (D+L)^-1 U,  S = L (D+U)^-1,  Y = (D+L)^-1 D (D+U)^-1   (eqs T, S, series)

whose limit is C^-1 by the recursion C^-1 = Y + T C^-1 S (eq recursive).
Sec. 2.2: the chains converge iff sp(T) < 1 and sp(S) < 1.
"""

from __future__ import annotations

import numpy as np


def split(C):
    """(L, D, U): strict lower triangle, diagonal, strict upper triangle."""
    C = np.asarray(C)
    return np.tril(C, -1), np.diag(np.diag(C)), np.triu(C, 1)


def operators(C):
    """(T, S, Y) of the demonstration, Sec. 2.1."""
    L, D, U = split(C)
    T = np.linalg.solve(D + L, U)
    S = L @ np.linalg.inv(D + U)
    Y = np.linalg.solve(D + L, D) @ np.linalg.inv(D + U)
    return T, S, Y


def expected_zw(C, k, z0=None, w0=None):
    """Exact E[z^(k) w^(k)dagger] after k sweeps from initial vectors z0, w0
    (default 0): sum_{m<k} T^m Y S^m + T^k z0 w0^dagger S^k (eqs zn, wn)."""
    T, S, Y = operators(C)
    n = T.shape[0]
    acc = np.zeros((n, n), dtype=np.result_type(T, S, Y, np.complex128))
    Tm = np.eye(n)
    Sm = np.eye(n)
    for _ in range(k):
        acc += Tm @ Y @ Sm
        Tm = Tm @ T
        Sm = S @ Sm
    if z0 is not None and w0 is not None:
        acc += Tm @ np.outer(z0, np.conj(w0)) @ Sm
    return acc


def spectral_radius(M):
    return float(np.max(np.abs(np.linalg.eigvals(M))))


def lattice_constant_phase_inverse_diag(L, k, a, b, theta, theta_p, dims=4):
    """Closed form for the translation-invariant lattice operator
    C = I - k sum_mu (a_mu e^{i theta_mu} shift_+mu + b_mu e^{-i theta'_mu} shift_-mu):
    plane waves e^{i p.x}, p_mu = 2 pi m / L, are eigenvectors with eigenvalue
    lambda(p) = 1 - k sum_mu (a_mu e^{i(theta_mu + p_mu)} + b_mu e^{-i(theta'_mu + p_mu)}).
    Returns (diagonal entry of C^-1, trace of C^-1)."""
    p = 2.0 * np.pi * np.arange(L) / L
    grids = np.meshgrid(*([p] * dims), indexing="ij")
    lam = np.ones(grids[0].shape, dtype=np.complex128)
    for mu in range(dims):
        lam -= k * (a[mu] * np.exp(1j * (theta[mu] + grids[mu]))
                    + b[mu] * np.exp(-1j * (theta_p[mu] + grids[mu])))
    tr = np.sum(1.0 / lam)
    return tr / L ** dims, tr


def dirac_free_trace(N, K, dims=4):
    """tr L^-1 of the free Wilson-Dirac matrix L = 1 + K sum_mu [(1 + gamma_mu)
    shift_+mu + (1 - gamma_mu) shift_-mu] on a periodic N^4 lattice.  Plane
    waves e^{i p.x}, p_mu = 2 pi m / N, block-diagonalise L into the 4 x 4
    matrices a(p) + i sum_mu b_mu(p) gamma_mu with a = 1 + 2K sum_mu cos p_mu
    and b_mu = 2K sin p_mu; the gamma anticommutation gives their inverse as
    (a - i b.gamma) / (a^2 + |b|^2), whose trace is 4a / (a^2 + |b|^2)."""
    p = 2.0 * np.pi * np.arange(N) / N
    grids = np.meshgrid(*([p] * dims), indexing="ij")
    a = 1.0 + 2.0 * K * sum(np.cos(g) for g in grids)
    b2 = 4.0 * K * K * sum(np.sin(g) ** 2 for g in grids)
    return float(np.sum(4.0 * a / (a * a + b2)))
