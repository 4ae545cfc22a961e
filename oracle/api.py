"""Entry points of the oracle: per-sample log P and the full estimate.

The limits a, b are given in integration order (already permuted).  The
factor is either a dense lower-triangular array or a TLR tuple
(diag, ranks, U, V).  Sample k (1-based) of shift s uses the lattice point
of lattice.py; nu = 0 selects the normal case, nu > 0 the Student-t case
(Section 2.2, Eq. 4: R = chi_nu^-1(w_0) / sqrt(nu) scales both limits).
"""

from __future__ import annotations

import math

import numpy as np

from . import estimate as est
from . import lattice, sov
from . import special as sf
from .factor import TLRRows


def rows_of(factor):
    if isinstance(factor, np.ndarray):
        return sov.DenseRows(factor)
    if isinstance(factor, (sov.DenseRows, TLRRows)):
        return factor
    diag, ranks, U, V = factor[:4]
    return TLRRows(diag, ranks, U, V)


class Lattice:
    """Generators and shift table for one problem (dimension n + 1)."""

    def __init__(self, n: int, M: int, seed: int):
        self.A = lattice.generators(n + 1)
        self.D = lattice.shifts(seed, M, n + 1)

    def points(self, s: int, ks) -> np.ndarray:
        return lattice.points(self.A, self.D[s], np.asarray(ks))


def sample_logp(factor, a, b, nu: float, seed: int, M: int, s: int, ks, lat=None):
    """log P of samples ks (1-based) of shift s."""
    rows = rows_of(factor)
    n = rows.n
    lat = lat or Lattice(n, M, seed)
    W = lat.points(s, ks)
    R = None if nu == 0 else sf.chi_inv(nu, W[0]) / math.sqrt(nu)
    return sov.sov_logp(rows, np.asarray(a, float), np.asarray(b, float), W[1:], R)


def probability(factor, a, b, nu: float, N: int, M: int, seed: int, chunk: int = 4096):
    """Full estimate over N samples x M shifts; returns (result dict, logp M x N)."""
    rows = rows_of(factor)
    lat = Lattice(rows.n, M, seed)
    logp = np.empty((M, N))
    for s in range(M):
        for k0 in range(1, N + 1, chunk):
            ks = np.arange(k0, min(k0 + chunk, N + 1))
            logp[s, ks - 1] = sample_logp(rows, a, b, nu, seed, M, s, ks, lat)
    return est.estimate(logp), logp
