"""Covariance, geometric order and the tile-low-rank Cholesky factor.

Section 3.2 (TLR as a practical representation): locations are indexed so
that index distance follows spatial distance; Section 3.3 / 3.4 (TLR
factorizations, TLR QMC): the factor is stored as dense diagonal tiles B_i
and off-diagonal tiles L_ij = U_ij V_ij^T truncated at a fixed absolute
tolerance.

Readings taken:

* geometric order: Morton (Z-order) of the locations quantised to 16 bits
  per axis over their bounding box, ties by original index (the paper uses
  HLIBpro's cardinality-balanced clustering, which is not available here);
* truncation: the factor is the exact dense Cholesky factor of the permuted
  covariance, and each off-diagonal tile keeps the singular values above
  ``tol`` (absolute, 2-norm), at most ``cap`` of them when cap > 0.  The
  paper compresses the covariance by ACA and truncates inside a TLR
  Cholesky; for a unit-variance kernel both keep every tile within the same
  absolute tolerance.
"""

from __future__ import annotations

import numpy as np


def exp_cov(xy: np.ndarray, beta: float, idx=None) -> np.ndarray:
    """Sigma_pq = exp(-|x_p - x_q| / beta) (exponential kernel, Section 3.2)."""
    p = xy if idx is None else xy[idx]
    d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
    return np.exp(-d / beta)


def _part1by1(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0xFFFF)
    out = np.zeros_like(v)
    for bit in range(16):
        out |= ((v >> np.uint64(bit)) & np.uint64(1)) << np.uint64(2 * bit)
    return out


def morton_order(xy: np.ndarray) -> np.ndarray:
    """Permutation (position -> location index) sorting locations in Z-order.

    q = floor((x - lo) / (hi - lo) * 65535 + 0.5) per axis; the key puts
    the bits of the first coordinate in the odd positions.
    """
    q = []
    for ax in range(2):
        x = xy[:, ax]
        lo, hi = float(np.min(x)), float(np.max(x))
        if hi > lo:
            q.append(np.floor((x - lo) / (hi - lo) * 65535.0 + 0.5).astype(np.uint64))
        else:
            q.append(np.zeros(len(x), dtype=np.uint64))
    key = (_part1by1(q[0]) << np.uint64(1)) | _part1by1(q[1])
    return np.argsort(key, kind="stable").astype(np.int32)


def tile_sizes(n: int, m: int) -> list[int]:
    r = (n + m - 1) // m
    return [min(m, n - i * m) for i in range(r)]


def tlr_from_dense(L: np.ndarray, m: int, tol: float, cap: int = 0):
    """Split a dense lower-triangular L into (diag, ranks, U, V, cap_hits)."""
    n = L.shape[0]
    sz = tile_sizes(n, m)
    r = len(sz)
    off = np.concatenate([[0], np.cumsum(sz)])
    diag = [np.tril(L[off[i]:off[i + 1], off[i]:off[i + 1]]).copy() for i in range(r)]
    ranks = np.zeros((r, r), dtype=np.int32)
    U, V = {}, {}
    hits = 0
    for i in range(r):
        for j in range(i):
            T = L[off[i]:off[i + 1], off[j]:off[j + 1]]
            P, s, Qt = np.linalg.svd(T, full_matrices=False)
            k = int(np.sum(s > tol))
            if cap > 0 and k > cap:
                k = cap
                hits += 1
            ranks[i, j] = k
            U[(i, j)] = P[:, :k] * s[:k]
            V[(i, j)] = Qt[:k, :].T.copy()
    return diag, ranks, U, V, hits


class TLRRows:
    """Row provider expanding a TLR factor to dense rows, one tile row at a time."""

    def __init__(self, diag, ranks, U, V):
        self.diag, self.ranks, self.U, self.V = diag, ranks, U, V
        sz = [d.shape[0] for d in diag]
        self.off = np.concatenate([[0], np.cumsum(sz)]).astype(np.int64)
        self.n = int(self.off[-1])
        self.blocks = [(int(self.off[i]), int(self.off[i + 1])) for i in range(len(sz))]

    def rows(self, i0: int, i1: int) -> np.ndarray:
        i = int(np.searchsorted(self.off, i0))
        out = np.zeros((i1 - i0, i1))
        for j in range(i):
            if self.ranks[i, j] > 0:
                out[:, self.off[j]:self.off[j + 1]] = self.U[(i, j)] @ self.V[(i, j)].T
        out[:, i0:i1] = np.tril(self.diag[i])
        return out

    def dense(self) -> np.ndarray:
        L = np.zeros((self.n, self.n))
        for (i0, i1) in self.blocks:
            L[i0:i1, :i1] = self.rows(i0, i1)
        return L


def tlr_factor(xy: np.ndarray, beta: float, perm: np.ndarray, m: int, tol: float,
               cap: int = 0):
    """Exponential-kernel covariance in order ``perm``, Cholesky, tile truncation."""
    S = exp_cov(xy, beta, perm)
    L = np.linalg.cholesky(S)
    return tlr_from_dense(L, m, tol, cap)
