"""Block reordering (Section 3.3, "Block reordering" algorithm) and its
iterative form that produces the Cholesky factor ("Block reordering during
Cholesky factorization").

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

The iterative form re-scores the remaining blocks at every elimination step
on the current (conditional) covariance and limits; the truncated means y_j
it conditions with are the univariate conditioning's means of the whitened
variables of block j, so the update a_i - L_ij y_j uses the factor's own
panel L_ij (the listing's Sigma_ij after its triangular solve).
"""

from __future__ import annotations

import numpy as np

from . import special as sf


def univariate_conditioning(S: np.ndarray, a: np.ndarray, b: np.ndarray, with_means: bool = False):
    """Returns (order, log p): the chosen order of the block and log of its
    score; with_means adds y, the truncated means of the whitened variables in
    that order."""
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
    if with_means:
        return order, logp, y
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


def iterative_block_reorder(S: np.ndarray, a: np.ndarray, b: np.ndarray, m: int, base: np.ndarray):
    """Block reordering during the Cholesky factorization.

    Returns (perm, L): perm[i] = original index at position i, and L the
    lower Cholesky factor of S[perm][:, perm].  ``S`` is in original
    indexing; ``base`` is the geometric order whose consecutive m-chunks are
    the blocks.  At step j the blocks j..(last full block) are scored by the
    univariate conditioning estimate on the current Schur complement and the
    current limits; the lowest score (lowest index on ties) is swapped into
    place and takes its within-block order; then the block is factored, the
    panel below is solved, the later limits are conditioned on the block's
    truncated means, and the Schur complement is updated.
    """
    base = np.asarray(base)
    n = len(base)
    A = np.array(S, dtype=np.float64)[np.ix_(base, base)]
    al = np.array(a, dtype=np.float64)[base]
    bl = np.array(b, dtype=np.float64)[base]
    perm = base.copy()
    L = np.zeros((n, n))
    r = (n + m - 1) // m
    nsort = r if n % m == 0 else r - 1

    def blk(j):
        return slice(j * m, min((j + 1) * m, n))

    def apply(pi, j0):
        """Reorder positions j0.. by pi (new position -> old position)."""
        nonlocal A, al, bl, perm, L
        idx = np.arange(n)
        idx[j0:] = j0 + pi
        A = A[np.ix_(idx, idx)]
        L = L[idx, :]
        al, bl, perm = al[idx], bl[idx], perm[idx]

    for j in range(r):
        j0 = j * m
        if j < nsort:
            scored = [univariate_conditioning(A[blk(l), blk(l)], al[blk(l)], bl[blk(l)]) for l in range(j, nsort)]
            t = j + int(np.argmin([lp for (_, lp) in scored]))
            if t != j:
                pi = np.arange(n - j0)
                bj, bt = np.arange(0, m), np.arange((t - j) * m, (t - j + 1) * m)
                pi[bj], pi[bt] = bt, bj
                apply(pi, j0)
        sj = blk(j)
        mj = sj.stop - sj.start
        order, _, y = univariate_conditioning(A[sj, sj], al[sj], bl[sj], with_means=True)
        pi = np.arange(n - j0)
        pi[:mj] = order
        apply(pi, j0)
        Ljj = np.linalg.cholesky(A[sj, sj])
        L[sj, sj] = Ljj
        rest = slice(sj.stop, n)
        if sj.stop < n:
            Lr = np.linalg.solve(Ljj, A[rest, sj].T).T  # A_rest,j Ljj^-T
            L[rest, sj] = Lr
            shift = Lr @ y
            al[rest] = al[rest] - shift
            bl[rest] = bl[rest] - shift
            A[rest, rest] = A[rest, rest] - Lr @ Lr.T
    return perm.astype(np.int32), L
