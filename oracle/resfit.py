"""FP64 numpy oracle of the residual-model regression (the Fig. 4b procedure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.

The paper fits the Fisk distribution to optical-flow residuals binned by the
observed flow magnitude, and then fits the laws of Eq. 6-7 to the per-bin
parameters: A(v) = a1 exp(a2 |v|), B(v) = b1 |v| + b2.  Reading used here:
  * residual x = |X - G|^2 (squared end-point error, the variable of Eq. 5),
    floored at x_floor; observed flow v = X; non-finite items are skipped;
  * bins of equal width over |v| in [0, v_max), items beyond are skipped;
  * per bin, a Fisk fit by moments of y = log x: the log of a Fisk variable is
    logistic with location log(alpha) and scale 1/beta, so
    log(alpha) = mean(y) and beta = pi / sqrt(3 var(y));
  * least squares weighted by the bin counts over the bins with at least
    min_count items: log(alpha_b) = log(a1) + a2 vbar_b and
    beta_b = b1 vbar_b + b2, vbar_b the bin's mean |v|.
"""
from __future__ import annotations

import numpy as np


def bin_stats(X, G, nbins, v_max, x_floor=1e-12):
    """Per-bin (count, sum |v|, sum y, sum y^2) of flows X, G [..., 2]."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 2)
    G = np.asarray(G, dtype=np.float64).reshape(-1, 2)
    ok = np.isfinite(X).all(axis=1) & np.isfinite(G).all(axis=1)
    X, G = X[ok], G[ok]
    v = np.sqrt((X * X).sum(axis=1))
    x = np.maximum(((X - G) ** 2).sum(axis=1), x_floor)
    y = np.log(x)
    b = np.floor(v * (nbins / v_max)).astype(np.int64)
    keep = (b >= 0) & (b < nbins)
    out = np.zeros((nbins, 4))
    for k in range(nbins):
        m = keep & (b == k)
        out[k] = [m.sum(), v[m].sum(), y[m].sum(), (y[m] ** 2).sum()]
    return out


def fit(stats, min_count=64):
    """(a1, a2, b1, b2) from per-bin statistics, and the per-bin (vbar, alpha, beta)."""
    n, sv, sy, syy = stats.T
    nn = np.maximum(n, 1)
    # bins with too few items, or with no spread (no finite Fisk shape), are left out
    use = (n >= min_count) & (syy / nn - (sy / nn) ** 2 > 0)
    vbar = sv[use] / n[use]
    mean = sy[use] / n[use]
    var = syy[use] / n[use] - mean ** 2
    beta = np.pi / np.sqrt(3.0 * var)
    w = np.sqrt(n[use])
    A = np.stack([np.ones_like(vbar), vbar], axis=1) * w[:, None]
    la1, a2 = np.linalg.lstsq(A, mean * w, rcond=None)[0]
    b2, b1 = np.linalg.lstsq(A, beta * w, rcond=None)[0]
    return (float(np.exp(la1)), float(a2), float(b1), float(b2)), np.stack([vbar, np.exp(mean), beta], axis=1)
