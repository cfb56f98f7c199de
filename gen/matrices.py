"""Matrix generators (data only).

Every generator is seeded and returns a :class:`CSR` with sorted, duplicate-free
column indices.  The shapes follow the paper's two workload families:

* a real non-symmetric, strictly diagonally dominant random sparse matrix
  (small dense-checkable case);
* a pedigree-structured real non-symmetric matrix whose off-diagonal pattern
  follows the asymmetric relationship-matrix rules of Example 1 (Sec. 3.1, the
  Wu-Schaeffer rules 2-4 with weight lambda) -- the real pedigree data and herd
  effects are not available, so animals, parents and matings are drawn at
  random;
* a complex non-hermitian nearest-neighbour operator on a periodic 4-D lattice,
  a random-phase stand-in for the lattice operator of Example 2 (Sec. 3.2).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """Compressed sparse rows: ``row_ptr`` int64[n+1], ``col`` int32[nnz],
    ``val`` float64[nnz] or complex128[nnz] (columns sorted within a row)."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.val)

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _from_coo(n, rows, cols, vals) -> CSR:
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return CSR(n=n, row_ptr=m.indptr.astype(np.int64), col=m.indices.astype(np.int32),
               val=np.ascontiguousarray(m.data))


def _set_dominant_diagonal(n, rows, cols, vals, factor):
    """Replace the diagonal by ``factor`` times the off-diagonal absolute row sum
    (1.0 for a row without off-diagonals) so that every row is strictly
    dominant."""
    off = rows != cols
    rows, cols, vals = rows[off], cols[off], vals[off]
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    rs = np.asarray(abs(m).sum(axis=1)).ravel()
    d = np.where(rs > 0, factor * rs, 1.0)
    coo = m.tocoo()
    r = np.concatenate([coo.row, np.arange(n)])
    c = np.concatenate([coo.col, np.arange(n)])
    v = np.concatenate([coo.data, d.astype(coo.data.dtype)])
    return _from_coo(n, r, c, v)


def random_dominant(n=200, offdiag_per_row=4, seed=1000, factor=1.5) -> CSR:
    """Real non-symmetric sparse matrix: per row ``offdiag_per_row`` distinct
    off-diagonal columns drawn uniformly without replacement, values U(-1, 1),
    diagonal = ``factor`` x off-diagonal absolute row sum."""
    rng = np.random.default_rng(seed)
    k = min(offdiag_per_row, n - 1)
    rows, cols = [], []
    for i in range(n):
        c = rng.choice(n - 1, size=k, replace=False)
        c = c + (c >= i)
        rows.append(np.full(k, i))
        cols.append(c)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = rng.uniform(-1.0, 1.0, size=rows.size)
    return _set_dominant_diagonal(n, rows, cols, vals, factor)


def pedigree(n=100_000, seed=1001, founders=0.05, lam=0.2, factor=1.5,
             jitter=(0.8, 1.2), symmetric=False) -> CSR:
    """Pedigree-shaped real non-symmetric matrix.

    Animals ``0 .. nf-1`` are founders (no parents); every later animal ``i``
    has a sire and a distinct dam drawn uniformly from ``[0, i)``.  For each
    animal with both parents known (delta = 2) the asymmetric relationship rules
    add ``-(1-lam) delta/2`` at (i,s), (i,d); ``-delta/2`` at (s,i), (d,i); and
    ``-delta/4`` at (s,d), (d,s) (duplicates summed).  Each stored off-diagonal
    is then multiplied by an independent U(jitter) factor, and the diagonal is
    set to ``factor`` x the off-diagonal absolute row sum.

    ``symmetric=True`` (needs lam = 0, where the rules are symmetric) draws one
    jitter factor per unordered pair {i, j}, giving a symmetric positive
    definite matrix (diagonally dominant, positive diagonal).
    """
    if symmetric and lam != 0.0:
        raise ValueError("a symmetric pedigree needs lam = 0")
    rng = np.random.default_rng(seed)
    nf = max(1, min(n, int(round(founders * n))))
    i = np.arange(nf, n, dtype=np.int64)
    if i.size:
        s = np.floor(rng.random(i.size) * i).astype(np.int64)
        d = np.floor(rng.random(i.size) * (i - 1)).astype(np.int64)
        # animals with index 1 have only one earlier animal: the dam equals the sire
        d = np.where(i > 1, d + (d >= s), s)
        two = s != d
        i, s, d = i[two], s[two], d[two]
    else:
        s = d = i
    delta = 2.0
    a2 = -(1.0 - lam) * delta / 2.0
    a3 = -delta / 2.0
    a4 = -delta / 4.0
    rows = np.concatenate([i, i, s, d, s, d])
    cols = np.concatenate([s, d, i, i, d, s])
    vals = np.concatenate([np.full(i.size, a2), np.full(i.size, a2),
                           np.full(i.size, a3), np.full(i.size, a3),
                           np.full(i.size, a4), np.full(i.size, a4)])
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    coo = m.tocoo()
    jit = rng.uniform(jitter[0], jitter[1], size=coo.data.size)
    if symmetric:
        key = np.minimum(coo.row, coo.col).astype(np.int64) * n + np.maximum(coo.row, coo.col)
        _, first, inv = np.unique(key, return_index=True, return_inverse=True)
        jit = jit[first][inv]
    return _set_dominant_diagonal(n, coo.row.astype(np.int64), coo.col.astype(np.int64),
                                  coo.data * jit, factor)


def lattice(L=16, k=0.1, seed=1002, constant_phase=False, dims=4) -> CSR:
    """Complex non-hermitian nearest-neighbour operator on a periodic
    ``L^dims`` lattice: ``C[x,x] = 1``, ``C[x,x+mu] = -k a_mu exp(i theta_{x,mu})``,
    ``C[x,x-mu] = -k b_mu exp(-i theta'_{x,mu})`` with theta, theta' ~ U(0, 2pi)
    per (site, direction) and a_mu, b_mu ~ U(0.8, 1.2) per direction.  With
    ``constant_phase`` every site shares theta_mu, theta'_mu (translation
    invariant, so the inverse has a closed form).  Site index
    ``x0 + L x1 + L^2 x2 + ...``."""
    if L < 3:
        raise ValueError("L >= 3 keeps the +mu and -mu neighbours distinct")
    rng = np.random.default_rng(seed)
    V = L ** dims
    a = rng.uniform(0.8, 1.2, size=dims)
    b = rng.uniform(0.8, 1.2, size=dims)
    if constant_phase:
        th = np.broadcast_to(rng.uniform(0, 2 * np.pi, size=dims), (V, dims))
        thp = np.broadcast_to(rng.uniform(0, 2 * np.pi, size=dims), (V, dims))
    else:
        th = rng.uniform(0, 2 * np.pi, size=(V, dims))
        thp = rng.uniform(0, 2 * np.pi, size=(V, dims))
    site = np.arange(V, dtype=np.int64)
    coords = [(site // L ** mu) % L for mu in range(dims)]
    rows = [site]
    cols = [site]
    vals = [np.ones(V, dtype=np.complex128)]
    for mu in range(dims):
        stride = L ** mu
        up = site + (((coords[mu] + 1) % L) - coords[mu]) * stride
        dn = site + (((coords[mu] - 1) % L) - coords[mu]) * stride
        rows += [site, site]
        cols += [up, dn]
        vals += [-k * a[mu] * np.exp(1j * th[:, mu]), -k * b[mu] * np.exp(-1j * thp[:, mu])]
    out = _from_coo(V, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    out.params = dict(L=L, k=k, a=a, b=b, theta=np.asarray(th[0]) if constant_phase else None,
                      theta_p=np.asarray(thp[0]) if constant_phase else None, dims=dims)
    return out


def dirac_gammas():
    """Euclidean Dirac matrices in the Dirac representation: gamma_4 =
    diag(1, 1, -1, -1) and gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] with the
    Pauli matrices sigma_k; hermitian, {gamma_mu, gamma_nu} = 2 delta_mu_nu.
    Order: gamma_1, gamma_2, gamma_3, gamma_4."""
    s = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
         np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
         np.array([[1, 0], [0, -1]], dtype=np.complex128)]
    z = np.zeros((2, 2), dtype=np.complex128)
    g = [np.block([[z, -1j * sk], [1j * sk, z]]) for sk in s]
    g.append(np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128))
    return g


def dirac(N=18, K=0.1, dims=4) -> CSR:
    """Free Wilson-Dirac fermion matrix of the paper's second example on a
    periodic N^dims lattice: L = 1 + K sum_mu [(1 + gamma_mu) shift_+mu +
    (1 - gamma_mu) shift_-mu], where (shift_+mu psi)_x = psi_{x + mu}.  Rank
    4 N^dims, 14 stored entries per row (identity, two per spatial hop, one per
    time hop since gamma_4 is diagonal).  Index = site + N^dims * spinor, site
    = x_1 + N x_2 + N^2 x_3 + N^3 x_4 (direction 4 is time)."""
    if dims != 4:
        raise ValueError("the Dirac matrices are 4 x 4: dims = 4")
    if N < 3:
        raise ValueError("N >= 3 keeps the +mu and -mu neighbours distinct")
    V = N ** dims
    g = dirac_gammas()
    site = np.arange(V, dtype=np.int64)
    rows, cols, vals = [np.arange(4 * V, dtype=np.int64)], [np.arange(4 * V, dtype=np.int64)], \
        [np.ones(4 * V, dtype=np.complex128)]
    for mu in range(dims):
        stride = N ** mu
        x = (site // stride) % N
        up = site + (((x + 1) % N) - x) * stride
        dn = site + (((x - 1) % N) - x) * stride
        for nb, sign in ((up, 1.0), (dn, -1.0)):
            block = np.eye(4, dtype=np.complex128) + sign * g[mu]
            for a in range(4):
                for b in range(4):
                    if block[a, b] != 0:
                        rows.append(site + a * V)
                        cols.append(nb + b * V)
                        vals.append(np.full(V, K * block[a, b], dtype=np.complex128))
    m = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(4 * V, 4 * V)).tocsr()
    m.sort_indices()
    return CSR(n=4 * V, row_ptr=m.indptr.astype(np.int64), col=m.indices.astype(np.int32),
               val=np.ascontiguousarray(m.data))


def batched_sizes(m=512, lo=1000, hi=50000, seed=1003):
    """Matrix orders drawn log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=m))).astype(np.int64)


def batched_pedigrees(m=512, lo=1000, hi=50000, seed=1003):
    """``m`` independent pedigree matrices of log-uniform order."""
    sizes = batched_sizes(m, lo, hi, seed)
    return [pedigree(int(nm), seed=seed * 7919 + j) for j, nm in enumerate(sizes)]


def surrogate_params(count, seed=1004):
    """Per-matrix generator parameters for the learned-surrogate workload:
    dominance factor U(1.2, 2.0), lambda U(0, 0.5), founder share U(2%, 20%)."""
    rng = np.random.default_rng(seed)
    return [dict(factor=float(rng.uniform(1.2, 2.0)), lam=float(rng.uniform(0.0, 0.5)),
                 founders=float(rng.uniform(0.02, 0.20)), seed=int(seed * 104729 + j))
            for j in range(count)]


def diag_matrix(d) -> CSR:
    d = np.asarray(d)
    n = d.size
    return CSR(n=n, row_ptr=np.arange(n + 1, dtype=np.int64), col=np.arange(n, dtype=np.int32),
               val=np.ascontiguousarray(d))


def from_dense(A, keep_zero_diagonal=True) -> CSR:
    A = np.asarray(A)
    n = A.shape[0]
    mask = A != 0
    if keep_zero_diagonal:
        mask |= np.eye(n, dtype=bool)
    r, c = np.nonzero(mask)
    return CSR(n=n, row_ptr=np.concatenate([[0], np.cumsum(mask.sum(axis=1))]).astype(np.int64),
               col=c.astype(np.int32), val=np.ascontiguousarray(A[r, c]))


def to_dense(m: CSR) -> np.ndarray:
    return m.to_scipy().toarray()


def round_values(m: CSR, dtype) -> CSR:
    """Copy of ``m`` whose values are rounded to ``dtype`` (float32/complex64)
    and promoted back to 64-bit: the exact matrix a 32-bit sweep works on."""
    v = m.val.astype(dtype).astype(np.complex128 if m.is_complex else np.float64)
    return CSR(n=m.n, row_ptr=m.row_ptr.copy(), col=m.col.copy(), val=v)


# Named workloads (matrix seed 1000 + index, noise seed 0x412107 + index).
WORKLOADS = {
    "tiny": dict(kind="random", n=200, offdiag=4, seed=1000, noise_seed=0x412107 + 0,
                 pairs=1, groups=1, burn_in=500, samples=20000, dtype="f64"),
    "pedigree": dict(kind="pedigree", n=100_000, seed=1001, noise_seed=0x412107 + 1,
                     pairs=4096, groups=64, burn_in=200, samples=2000, dtype="f32",
                     block=256),
    "lattice": dict(kind="lattice", L=16, k=0.1, seed=1002, noise_seed=0x412107 + 2,
                    pairs=1024, groups=32, burn_in=100, samples=2000, dtype="c64"),
    "batched": dict(kind="batched", m=512, lo=1000, hi=50000, seed=1003,
                    noise_seed=0x412107 + 3, pairs=64, groups=16, burn_in=200,
                    samples=2000, dtype="f32", block=128),
    "surrogate": dict(kind="surrogate", train=2000, train_n=20000, eval_n=1_000_000,
                      seed=1004, noise_seed=0x412107 + 4),
    "dirac": dict(kind="dirac", N=18, K=0.1, noise_seed=0x412107 + 5, pairs=1024, groups=32,
                  rel_se=1e-5, dtype="c64"),
}
