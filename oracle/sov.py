"""Dense separation-of-variables integrand in log space.

Follows Eq. 2 of Section 2.1 and the "QMC for MVN probabilities" algorithm,
with two readings of that algorithm's listing:

* the division uses the Cholesky diagonal l_ii (the listing writes C_ii;
  Eq. 2 divides by l_ii);
* the quantile argument is d_i + w_i (e_i - d_i) as in Eq. 2 (the listing
  drops the d_i term, which is zero only when a_i = -inf).

The Student-t form (Section 2.2, Eq. 4 and the "mvt" algorithm built on it)
scales both limits by R = chi_nu^-1(w_0) / sqrt(nu) and then runs the same
recursion; TLR factors (Section 3.4) enter as their dense rows.

Log space (the paper is silent; its likelihoods reach 1e-40 and below): the
running product P is kept as log P.  Where a_i' > 0 the recursion uses the
complement CDFs, Phi(-a') - Phi(-b'), so that upper-tail intervals keep
their precision; the value of the integrand is unchanged.  Where the
interval probability is below ``special.TINY`` it is formed from log Phi.
An interval of probability exactly zero ends the sample: log P = -inf and
its remaining y are set to zero.
"""

from __future__ import annotations

import numpy as np

from . import special as sf


class DenseRows:
    """Row provider for an explicit dense lower-triangular factor L."""

    def __init__(self, L: np.ndarray, block: int = 1024):
        self.L = np.asarray(L, dtype=np.float64)
        self.n = self.L.shape[0]
        self.blocks = [(i, min(i + block, self.n)) for i in range(0, self.n, block)]

    def rows(self, i0: int, i1: int) -> np.ndarray:
        return self.L[i0:i1, :i1]


def _logdiffexp(x, y):
    """log(exp(x) - exp(y)) for x >= y."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return x + np.log1p(-np.exp(y - x))


def _step(ah, bh, w):
    """One variable: returns (log Delta, y) for conditional limits (ah, bh)."""
    lower = ah <= 0.0
    # Direct CDFs where a' <= 0, complements where a' > 0.
    lo = np.where(lower, ah, -bh)
    hi = np.where(lower, bh, -ah)
    d = sf.Phi(lo)
    e = sf.Phi(hi)
    delta = e - d
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.where(lower, d + w * delta, e - w * delta)
        y = sf.Phi_inv(u)
        log_delta = np.log(delta)
    small = delta <= sf.TINY
    if np.any(small):
        ld = sf.log_Phi(lo[small])
        le = sf.log_Phi(hi[small])
        ldel = _logdiffexp(le, ld)
        ws = w[small]
        lws = np.log(ws)
        low_s = lower[small]
        with np.errstate(divide="ignore", invalid="ignore"):
            lu = np.where(low_s, np.logaddexp(ld, lws + ldel), _logdiffexp(le, lws + ldel))
        log_delta[small] = ldel
        y[small] = sf.Phi_inv_log(lu)
    y = np.where(lower, y, -y)
    dead = ~(log_delta > -np.inf)
    log_delta = np.where(dead, -np.inf, log_delta)
    y = np.where(dead, 0.0, y)
    return log_delta, y


def sov_logp(rows, a: np.ndarray, b: np.ndarray, W: np.ndarray, R=None) -> np.ndarray:
    """log P for each column of W (n x S points, coordinates 1..n).

    ``rows`` gives the dense lower-triangular factor by blocks of rows;
    a, b are the limits in integration order; R (length S) scales them
    (Student-t), None for the normal case.
    """
    n, S = W.shape
    Y = np.zeros((n, S))
    logp = np.zeros(S)
    Rv = np.ones(S) if R is None else np.asarray(R, dtype=np.float64)
    for (i0, i1) in rows.blocks:
        Lb = rows.rows(i0, i1)
        for i in range(i0, i1):
            li = Lb[i - i0]
            s = li[:i] @ Y[:i] if i > 0 else np.zeros(S)
            lii = li[i]
            with np.errstate(invalid="ignore"):
                ah = (Rv * a[i] - s) / lii
                bh = (Rv * b[i] - s) / lii
            ld, y = _step(ah, bh, W[i])
            logp += ld
            Y[i] = y
    return logp
