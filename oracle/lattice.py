"""Richtmyer lattice points with random shifts, exactly, in Q0.64.

Section 2.1 (remark after the MVN algorithm) and Section 3.4 name the
Richtmyer rule without its constants.  Reading taken here (Richtmyer 1951):
coordinate c uses alpha_c = frac(sqrt(p_{c+1})), with p_1 = 2, p_2 = 3, ...
the consecutive primes.  Coordinate 0 feeds the chi radius of the Student-t
form (Eq. 4, "mvt" algorithm: (w_0, w)); coordinates 1..n are the variables
in integration order.  Sample k = 1..N of shift s is

    w_{k,c} = frac(k * alpha_c + Delta_{s,c}),

computed exactly in 64-bit fixed point: A_c = floor(alpha_c * 2^64),
W = (k * A_c + D_{s,c}) mod 2^64, w = ((W >> 12) + 1/2) * 2^-52, which lies
in [2^-53, 1 - 2^-53] and is an exact double.

Shifts D_{s,c} are the outputs of one SplitMix64 stream (Steele, Lea and
Flood 2014) with state = seed, drawn s-major, c-minor.
"""

from __future__ import annotations

import math

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def primes(count: int) -> list[int]:
    """The first ``count`` primes (sieve of Eratosthenes)."""
    if count <= 0:
        return []
    lim = max(16, int(count * (math.log(count + 1) + math.log(math.log(count + 2)) + 3)))
    while True:
        sieve = bytearray([1]) * (lim + 1)
        sieve[0:2] = b"\x00\x00"
        for q in range(2, int(lim ** 0.5) + 1):
            if sieve[q]:
                sieve[q * q::q] = bytearray(len(range(q * q, lim + 1, q)))
        ps = [i for i in range(lim + 1) if sieve[i]]
        if len(ps) >= count:
            return ps[:count]
        lim *= 2


def generators(dim: int) -> np.ndarray:
    """A_c = floor(frac(sqrt(p_{c+1})) * 2^64), c = 0..dim-1, as uint64.

    floor(sqrt(p) * 2^64) is the integer square root of p * 2^128; its low
    64 bits are the fraction.
    """
    return np.array([math.isqrt(p << 128) & _MASK for p in primes(dim)],
                    dtype=np.uint64)


def splitmix64(state: int, count: int) -> list[int]:
    """First ``count`` outputs of SplitMix64 with the given state (Python ints)."""
    out = []
    s = state & _MASK
    for _ in range(count):
        s = (s + _GAMMA) & _MASK
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        out.append(z ^ (z >> 31))
    return out


def shifts(seed: int, n_shifts: int, dim: int) -> np.ndarray:
    """D[s, c] (uint64), s = 0..M-1, c = 0..dim-1, s-major from one stream."""
    return np.array(splitmix64(seed, n_shifts * dim), dtype=np.uint64).reshape(n_shifts, dim)


def points(A: np.ndarray, D_s: np.ndarray, k: np.ndarray, cols=None) -> np.ndarray:
    """w[c, j] for samples k[j] of one shift: ((k*A_c + D_c mod 2^64) >> 12 + 1/2) 2^-52.

    ``cols`` selects coordinates (default: all).  numpy's uint64 product and
    sum wrap modulo 2^64, which is the definition above.
    """
    if cols is not None:
        A = A[cols]
        D_s = D_s[cols]
    kk = np.asarray(k, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        W = kk * A[:, None] + D_s[:, None]
    return ((W >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)
