"""Oracle for the learned surrogate of diag(C^-1) (test infrastructure only).

Target.  With C = D (I + M), M = D^-1 R (R = off-diagonal part), the Neumann
series gives d_i (C^-1)_ii = sum_k (-1)^k (M^k)_ii = 1 + (M^2)_ii - (M^3)_ii + ...
The surrogate predicts y_i = c_ii (C^-1)_ii from local features of row i;
labels come from the Monte Carlo estimates of eq (1/C).

Features (32 per row, float): see FEATURES below; every one is a local
function of the rows and columns within two hops of i.

MLP 32 -> 128 -> 128 -> 1 with GELU (erf form); the GPU runs it with bf16
operands and fp32 accumulation.  `mlp_grads(..., bf16=True)` rounds operands
to bf16 at exactly the points the GPU does (round to nearest even), computing
everything else in float64, so the two gradients agree to fp32 accumulation
order; with `bf16=False` it is the plain float64 network (pinned by finite
differences in the tests).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.special import erf

NF = 32
H = 128

FEATURES = [
    "log|c_ii|",
    "row abs sum / |c_ii|",
    "column abs sum / |c_ii|",
    "row off-diagonal count / 8",
    "column off-diagonal count / 8",
    "(M^2)_ii  (2-cycles)",
    "(M^3)_ii  (3-cycles)",
    "sum_j |m_ij| |m_ji|",
    "sum_j m_ij^2",
    "signed row sum / c_ii",
    "signed column sum / c_ii",
    "neighbours' row ratio: mean", "max", "min", "std",
    "neighbours' log(|c_jj|/|c_ii|): mean", "max", "min", "std",
    "neighbours' (M^2)_jj: mean", "max",
    "neighbours' column ratio: mean", "max",
    "neighbours' (M^3)_jj: mean",
    "neighbour count (merged pattern) / 8",
    "Neumann-2 estimate 1 + (M^2)_ii",
    "Neumann-3 estimate 1 + (M^2)_ii - (M^3)_ii",
    "row ratio squared",
    "(M^2)_ii squared",
    "(M^2)_ii x row ratio",
    "neighbours' row ratio: sum of squares / 8",
    "constant 1",
]
assert len(FEATURES) == NF


def features(m):
    """[n][32] float64 features of matrix m (gen.CSR, real)."""
    A = m.to_scipy().tocsr().astype(np.float64)
    n = m.n
    d = A.diagonal()
    R = (A - sp.diags(d)).tocsr()
    R.eliminate_zeros()
    Dinv = sp.diags(1.0 / d)
    M = (Dinv @ R).tocsr()
    ad = np.abs(d)
    absR = abs(R)
    f = np.zeros((n, NF))
    f[:, 0] = np.log(ad)
    f[:, 1] = np.asarray(absR.sum(axis=1)).ravel() / ad
    f[:, 2] = np.asarray(absR.sum(axis=0)).ravel() / ad
    f[:, 3] = np.diff(R.indptr) / 8.0
    f[:, 4] = np.diff(R.tocsc().indptr) / 8.0
    MT = M.T.tocsr()
    m2 = np.asarray(M.multiply(MT).sum(axis=1)).ravel()
    M2 = (M @ M).tocsr()
    m3 = np.asarray(M2.multiply(MT).sum(axis=1)).ravel()
    f[:, 5] = m2
    f[:, 6] = m3
    f[:, 7] = np.asarray(abs(M).multiply(abs(MT)).sum(axis=1)).ravel()
    f[:, 8] = np.asarray(M.multiply(M).sum(axis=1)).ravel()
    f[:, 9] = np.asarray(R.sum(axis=1)).ravel() / d
    f[:, 10] = np.asarray(R.sum(axis=0)).ravel() / d
    # merged neighbour pattern (row i or column i of C, j != i)
    S = ((abs(R) + abs(R).T) > 0).astype(np.float64).tocsr()
    cnt = np.diff(S.indptr).astype(np.float64)

    def nstats(v):
        # mean, max, min and population std (two passes: sum of squared deviations)
        s1 = np.asarray(S @ v).ravel()
        mean = np.where(cnt > 0, s1 / np.maximum(cnt, 1), 0.0)
        mx = np.zeros(n)
        mn = np.zeros(n)
        var = np.zeros(n)
        for i in range(n):
            idx = S.indices[S.indptr[i]:S.indptr[i + 1]]
            if idx.size:
                mx[i] = v[idx].max()
                mn[i] = v[idx].min()
                var[i] = np.sum((v[idx] - mean[i]) ** 2) / idx.size
        return mean, mx, mn, np.sqrt(var)

    mean, mx, mn, sd = nstats(f[:, 1])
    f[:, 11], f[:, 12], f[:, 13], f[:, 14] = mean, mx, mn, sd
    # log(|c_jj| / |c_ii|) = log|c_jj| - log|c_ii|
    lg = f[:, 0]
    mean, mx, mn, sd = nstats(lg)
    f[:, 15] = np.where(cnt > 0, mean - lg, 0.0)
    f[:, 16] = np.where(cnt > 0, mx - lg, 0.0)
    f[:, 17] = np.where(cnt > 0, mn - lg, 0.0)
    f[:, 18] = sd
    mean, mx, _, _ = nstats(m2)
    f[:, 19], f[:, 20] = mean, mx
    mean, mx, _, _ = nstats(f[:, 2])
    f[:, 21], f[:, 22] = mean, mx
    mean, _, _, _ = nstats(m3)
    f[:, 23] = mean
    f[:, 24] = cnt / 8.0
    f[:, 25] = 1.0 + m2
    f[:, 26] = 1.0 + m2 - m3
    f[:, 27] = f[:, 1] ** 2
    f[:, 28] = m2 ** 2
    f[:, 29] = m2 * f[:, 1]
    f[:, 30] = np.asarray(S @ (f[:, 1] ** 2)).ravel() / 8.0
    f[:, 31] = 1.0
    return f


# ----------------------------------------------------------------- the MLP --
def bf16(x):
    """Round float values to bfloat16 (nearest even) and return them as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_prime(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def init_params(seed):
    """Same initialisation as the library: W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)),
    biases 0, output bias 1 (y is close to 1)."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.uniform(-1, 1, (NF, H)) / np.sqrt(NF),
        "b1": np.zeros(H),
        "W2": rng.uniform(-1, 1, (H, H)) / np.sqrt(H),
        "b2": np.zeros(H),
        "w3": rng.uniform(-1, 1, H) / np.sqrt(H),
        "b3": np.array([1.0]),
    }


def mlp_forward(p, X, bf16_ops=True):
    r = bf16 if bf16_ops else (lambda v: np.asarray(v, dtype=np.float64))
    z1 = r(X) @ r(p["W1"]) + p["b1"]
    h1 = gelu(z1)
    z2 = r(h1) @ r(p["W2"]) + p["b2"]
    h2 = gelu(z2)
    out = h2 @ p["w3"] + p["b3"][0]
    return out, (z1, h1, z2, h2)


def mlp_loss(p, X, y, w, bf16_ops=True, denom=None):
    """Weighted MSE sum_r w_r (out_r - y_r)^2 / denom (default: sum w)."""
    out, _ = mlp_forward(p, X, bf16_ops)
    denom = np.sum(w) if denom is None else denom
    return float(np.sum(w * (out - y) ** 2) / denom)


def mlp_grads(p, X, y, w, bf16_ops=True, denom=None):
    """Gradients of mlp_loss (backpropagation through the three layers)."""
    r = bf16 if bf16_ops else (lambda v: np.asarray(v, dtype=np.float64))
    out, (z1, h1, z2, h2) = mlp_forward(p, X, bf16_ops)
    denom = np.sum(w) if denom is None else denom
    dout = 2.0 * w * (out - y) / denom
    g = {}
    g["w3"] = h2.T @ dout
    g["b3"] = np.array([dout.sum()])
    dz2 = (dout[:, None] * p["w3"][None, :]) * gelu_prime(z2)
    g["W2"] = r(h1).T @ r(dz2)
    g["b2"] = dz2.sum(axis=0)
    dh1 = r(dz2) @ r(p["W2"]).T
    dz1 = dh1 * gelu_prime(z1)
    g["W1"] = r(X).T @ r(dz1)
    g["b1"] = dz1.sum(axis=0)
    return g


def flatten(p):
    """Parameters in the library's order: W1 (input-major), b1, W2, b2, w3, b3."""
    return np.concatenate([np.ravel(p[k]) for k in ORDER])


def unflatten(v):
    v = np.asarray(v, dtype=np.float64)
    out, o = {}, 0
    for k in ORDER:
        size = int(np.prod(SHAPES[k]))
        out[k] = v[o:o + size].reshape(SHAPES[k]).copy()
        o += size
    return out


ORDER = ["W1", "b1", "W2", "b2", "w3", "b3"]
SHAPES = {"W1": (NF, H), "b1": (H,), "W2": (H, H), "b2": (H,), "w3": (H,), "b3": (1,)}
N_PARAMS = sum(int(np.prod(v)) for v in SHAPES.values())


def normalize(X, mean, inv_std):
    """(x - mean) * inv_std, each operation rounded to float32 as the device does."""
    X = np.asarray(X, dtype=np.float32)
    return ((X - np.asarray(mean, np.float32)) * np.asarray(inv_std, np.float32)).astype(np.float64)


def fit_normalization(X):
    """Column means and inverse population standard deviations of the float32
    features (fp64 sums), 1 for a constant column; returned as float32."""
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    mean = X.mean(axis=0)
    var = ((X - mean) ** 2).mean(axis=0)
    inv = np.where(var > 1e-12, 1.0 / np.sqrt(np.where(var > 1e-12, var, 1.0)), 1.0)
    return mean.astype(np.float32), inv.astype(np.float32)


def label_weights(y_se, eps=1e-6):
    """Loss weights 1 / (se^2 + eps), scaled to mean 1."""
    raw = 1.0 / (np.asarray(y_se, np.float64) ** 2 + eps)
    return raw * (raw.size / raw.sum())


def batch_rows(seed, step, N, R):
    """Rows of training step `step` (1-based): floor(x N / 2^64) with x = (o0 << 32) | o1
    of the Philox4x32-10 block, key (seed lo, seed hi), counter (r, step, 0x5EED, 0xA11CE)."""
    from . import philox4x32_10
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    rows = np.empty(R, dtype=np.int64)
    for r in range(R):
        o = philox4x32_10((r, step, 0x5EED, 0xA11CE), (k0, k1))
        x = (int(o[0]) << 32) | int(o[1])
        rows[r] = (x * N) >> 64
    return rows


def adam_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba, 2015) with bias correction; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[:] = beta1 * m + (1 - beta1) * g[k]
        v[:] = beta2 * v + (1 - beta2) * g[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


# ---------------------------------------------------------------- the gate --
def gate_edges(v, bins):
    """Quantile edges of one feature: sorted values at floor(k N / bins), k = 1..bins-1."""
    v = np.sort(np.asarray(v, dtype=np.float64))
    N = v.size
    return np.array([v[(k * N) // bins] for k in range(1, bins)])


def gate_bin(edges, x):
    """Number of edges <= x."""
    return np.searchsorted(edges, np.asarray(x, dtype=np.float64), side="right")


def chi2_lower_quantile(k, z):
    """Wilson and Hilferty's (1931) normal approximation of the chi-square
    distribution with k degrees of freedom: (X / k)^(1/3) is close to normal
    with mean 1 - 2/(9k) and variance 2/(9k), so the quantile at standard
    normal value -z is k (1 - 2/(9k) - z sqrt(2/(9k)))^3 (floored at 1e-3)."""
    c = 2.0 / (9.0 * k)
    return max(k * (1.0 - c - z * np.sqrt(c)) ** 3, 1e-3)


def gate_fit(X, pred, y, y_se, fa, fb, bins, min_rows, tol, ucb_z=0.0):
    """Validated relative error per (feature a, feature b) bin: sqrt(max(sum r^2 - sum s^2, 0) / count)
    with r = (pred - y) / y and s = y_se / y (the label noise is removed from the observed spread);
    with ucb_z > 0 the count is replaced by the chi-square lower quantile above, which turns the
    error into an upper confidence bound; a bin needs the sampler when it has fewer than min_rows
    rows or that error exceeds tol."""
    X = np.asarray(X, dtype=np.float32)
    ea = gate_edges(X[:, fa], bins)
    eb = gate_edges(X[:, fb], bins)
    b = gate_bin(ea, X[:, fa]) * bins + gate_bin(eb, X[:, fb])
    r = (np.asarray(pred, np.float64) - y) / y
    s = np.asarray(y_se, np.float64) / y
    cnt = np.zeros(bins * bins, dtype=np.int64)
    r2 = np.zeros(bins * bins)
    s2 = np.zeros(bins * bins)
    for i in range(X.shape[0]):
        cnt[b[i]] += 1
        r2[b[i]] += r[i] * r[i]
        s2[b[i]] += s[i] * s[i]
    err = np.full(bins * bins, np.inf)
    for b in range(bins * bins):
        if cnt[b] > 0:
            q = chi2_lower_quantile(float(cnt[b]), ucb_z) if ucb_z > 0 else float(cnt[b])
            err[b] = np.sqrt(max(r2[b] - s2[b], 0.0) / q)
    fallback = (cnt < min_rows) | ~(err <= tol)
    xa = X[:, fa].astype(np.float64)
    xb = X[:, fb].astype(np.float64)
    return {"edges_a": ea, "edges_b": eb, "err": err, "count": cnt, "fallback": fallback,
            "fa": fa, "fb": fb, "bins": bins,
            "range_a": (xa.min(), xa.max()), "range_b": (xb.min(), xb.max())}


def gate_apply(g, X):
    """1 where a row's bin needs the sampler, where a binning feature is not a
    number, or where it lies outside the range the validation rows covered
    (the outer bins are open-ended: such a row has no validated error)."""
    X = np.asarray(X, dtype=np.float32)
    xa = X[:, g["fa"]].astype(np.float64)
    xb = X[:, g["fb"]].astype(np.float64)
    b = gate_bin(g["edges_a"], xa) * g["bins"] + gate_bin(g["edges_b"], xb)
    out = g["fallback"][b].astype(np.uint8)
    (la, ha), (lb, hb) = g["range_a"], g["range_b"]
    inside = (xa >= la) & (xa <= ha) & (xb >= lb) & (xb <= hb)   # False for NaN
    out[~inside] = 1
    return out
