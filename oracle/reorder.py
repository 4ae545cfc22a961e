"""Block reordering (Section 3.3, "Block reordering" algorithm).

Each size-m block l of variables (consecutive in the geometric order) gets
a score p[l] ~ Phi_m(a_l, b_l; Sigma_ll) from the univariate conditioning
method (Trinh and Genz 2015, cited in Section 3.3): one pass of a Cholesky
factorization that at each step picks the remaining variable with the
smallest conditional interval probability, then conditions the others on
the truncated mean of the chosen one.  The blocks are then put in ascending
order of p by selection with swaps, as the algorithm lists it.

Readings taken:

* the abstract and Section 3.1 say variables are reordered between and
  within blocks; the listing shows only the block swaps.  Within each block
  the variables take the order the univariate conditioning picked;
* ties in either argmin go to the lowest current index;
* a ragged last block (n not a multiple of m) stays last;
* the Student-t case scores with unscaled limits (R = 1).
"""

from __future__ import annotations

import numpy as np

from . import special as sf


def univariate_conditioning(S: np.ndarray, a: np.ndarray, b: np.ndarray):
    """Returns (order, log p): the chosen order of the block and log of its score."""
    m = len(a)
    S = np.array(S, dtype=np.float64, copy=True)
    a = np.array(a, dtype=np.float64, copy=True)
    b = np.array(b, dtype=np.float64, copy=True)
    order = np.arange(m)
    L = np.zeros((m, m))
    y = np.zeros(m)
    logp = 0.0
    for i in range(m):
        rest = np.arange(i, m)
        s = L[rest, :i] @ y[:i]
        var = np.diag(S)[rest] - np.sum(L[rest, :i] ** 2, axis=1)
        sd = np.sqrt(np.maximum(var, 0.0))
        with np.errstate(invalid="ignore", divide="ignore"):
            at = (a[rest] - s) / sd
            bt = (b[rest] - s) / sd
        prob = sf.Phi(bt) - sf.Phi(at)
        js = i + int(np.argmin(prob))
        if js != i:
            S[[i, js], :] = S[[js, i], :]
            S[:, [i, js]] = S[:, [js, i]]
            L[[i, js], :] = L[[js, i], :]
            a[[i, js]] = a[[js, i]]
            b[[i, js]] = b[[js, i]]
            order[[i, js]] = order[[js, i]]
        lii = sd[js - i]
        L[i, i] = lii
        if i + 1 < m:
            L[i + 1:, i] = (S[i + 1:, i] - L[i + 1:, :i] @ L[i, :i]) / lii
        al, bl = at[js - i], bt[js - i]
        pl = prob[js - i]
        if pl > 0:
            y[i] = (sf.phi(al) - sf.phi(bl)) / pl
            logp += float(np.log(pl))
        else:
            y[i] = bl if np.isfinite(bl) else (al if np.isfinite(al) else 0.0)
            logp = -np.inf
    return order, logp


def block_reorder(S: np.ndarray, a: np.ndarray, b: np.ndarray, m: int,
                  base: np.ndarray) -> np.ndarray:
    """Permutation (position -> original index) after block reordering.

    ``S`` is the covariance in original indexing, ``base`` the geometric
    order whose consecutive m-chunks are the blocks.
    """
    n = len(base)
    blocks = [np.asarray(base[i:min(i + m, n)]) for i in range(0, n, m)]
    nsort = len(blocks) if n % m == 0 else len(blocks) - 1
    scored = []
    for blk in blocks:
        order, lp = univariate_conditioning(S[np.ix_(blk, blk)], a[blk], b[blk])
        scored.append((blk[order], lp))
    p = [lp for (_, lp) in scored]
    for j in range(nsort):
        jt = j + int(np.argmin(p[j:nsort]))
        if jt != j:
            p[j], p[jt] = p[jt], p[j]
            scored[j], scored[jt] = scored[jt], scored[j]
    return np.concatenate([blk for (blk, _) in scored]).astype(np.int32)
