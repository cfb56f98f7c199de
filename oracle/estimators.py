"""Monte Carlo error estimates for the oracle (test infrastructure only).

The paper computes the standard error of a serially correlated chain from an
effective sample size (Sec. 2.3, citing Geyer 1992) and reports
``SE = sqrt(Var / N_eff)`` (Tables 2, 4, 5).  Two estimators are used:

* ``geyer_ips`` -- Geyer's initial positive sequence on one scalar series;
* ``cluster_estimate`` -- ratio estimator over independent clusters (groups of
  independent chain pairs, or consecutive time batches of one chain).
"""

from __future__ import annotations

import numpy as np


def _ips_real(x):
    x = np.asarray(x, dtype=np.float64)
    S = x.size
    xc = x - x.mean()
    g0 = float(xc @ xc) / S
    sig2 = -g0
    m = 0
    while 2 * m + 1 < S:
        ga = float(xc[: S - 2 * m] @ xc[2 * m:]) / S
        gb = float(xc[: S - 2 * m - 1] @ xc[2 * m + 1:]) / S
        pair_sum = ga + gb
        if pair_sum <= 0.0:
            break
        sig2 += 2.0 * pair_sum
        m += 1
    if sig2 <= 0.0:
        sig2 = g0
    return g0, sig2


def geyer_ips(x):
    """Mean of series ``x`` with Geyer's initial-positive-sequence error.

    gamma_t = (1/S) sum_k (x_k - xbar)(x_{k+t} - xbar);  Gamma_m = gamma_2m +
    gamma_2m+1, summed while positive;  sigma^2 = -gamma_0 + 2 sum Gamma_m;
    N_eff = S gamma_0 / sigma^2;  SE = sqrt(gamma_0 / N_eff).  A complex series
    is treated per component, SE = sqrt(SE_re^2 + SE_im^2).
    Returns dict(mean, var, n_eff, se)."""
    x = np.asarray(x)
    S = x.size
    if S < 2:
        return dict(mean=x.mean() if S else np.nan, var=np.nan, n_eff=np.nan, se=np.nan)
    parts = [x.real, x.imag] if np.iscomplexobj(x) else [x]
    g0 = sig2 = 0.0
    for comp in parts:
        a, b = _ips_real(comp)
        g0 += a
        sig2 += b
    se = np.sqrt(sig2 / S)
    n_eff = S * g0 / sig2 if sig2 > 0 else np.nan
    return dict(mean=x.mean(), var=g0, n_eff=n_eff, se=se)


def cluster_estimate(sums, counts):
    """Estimate and standard error from cluster sums.

    ``sums[c, ...]`` is the sum of the per-term values in cluster ``c`` and
    ``counts[c]`` its number of terms.  est = sum_c sums_c / sum_c counts_c;
    Var(est) = nc/(nc-1) sum_c (sums_c - counts_c est)^2 / (sum counts)^2 per
    real component; SE = sqrt(Var_re + Var_im).  Clusters without terms are
    ignored; fewer than two clusters give NaN."""
    sums = np.asarray(sums)
    counts = np.asarray(counts, dtype=np.float64)
    keep = counts > 0
    S = sums[keep]
    w = counts[keep]
    tot = w.sum()
    shape = (-1,) + (1,) * (S.ndim - 1)
    est = S.sum(axis=0) / tot
    nc = int(keep.sum())
    if nc < 2:
        return est, np.full(est.shape, np.nan)
    dev = S - w.reshape(shape) * est
    var = (dev.real ** 2).sum(axis=0) + (dev.imag ** 2).sum(axis=0)
    var = var * nc / (nc - 1) / tot ** 2
    return est, np.sqrt(var)
