"""Workload definitions and seeded draws (inputs only).

Every random number here comes from SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): output i
(0-based) of the stream with state ``s`` is mix(s + (i+1)*gamma).  The
stream is counter based, so any output can be drawn without the ones before.

The workloads follow the paper's simulation setting (Section 4: locations in
the unit square, exponential covariance exp(-|h|/beta), lower limits -inf)
with the concrete sizes of the benchmark configurations listed in CONFIGS.
The paper perturbs its grid; these workloads use the regular grid
x = (i/(g-1), j/(g-1)).
"""

from __future__ import annotations

import math

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(state: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream with ``state``."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(state & 0xFFFFFFFFFFFFFFFF) + idx * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(state: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1): the top 53 bits of each output times 2^-53."""
    x = splitmix64(state, count, start)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def grid_xy(g: int) -> np.ndarray:
    """g*g locations of the regular grid on the unit square, row-major (i, j)."""
    t = np.arange(g, dtype=np.float64) / (g - 1)
    xi, xj = np.meshgrid(t, t, indexing="ij")
    return np.stack([xi.ravel(), xj.ravel()], axis=1)


def upper_limits_uniform(n: int, seed: int, hi: float = 4.0) -> np.ndarray:
    """b_i iid U(0, hi), attached to the locations in grid order."""
    return hi * uniform01(seed, n)


# Benchmark configurations: sizes from the workload specification, seeds
# seed_b = 2003 + id (limits) and seed_shift = 11183 + id (random shifts).
CONFIGS = {
    1: dict(name="dense-mvn-n256", g=16, beta=0.1, m=256, tol=0.0, cap=0,
            reorder=False, nu=0.0, N=10_000, M=10, precision=0),
    2: dict(name="tlr-mvn-n4096", g=64, beta=0.1, m=64, tol=1e-5, cap=32,
            reorder=True, nu=0.0, N=20_000, M=10, precision=0),
    3: dict(name="tlr-mvt-n16384", g=128, beta=0.3, m=256, tol=1e-5, cap=0,
            reorder=False, nu=7.0, N=40_000, M=10, precision=1),
    4: dict(name="tlr-mvn-n65536", g=256, beta=0.1, m=512, tol=1e-5, cap=64,
            reorder=True, nu=0.0, N=20_000, M=10, precision=1),
}


def config(cid: int) -> dict:
    """Concrete inputs of configuration ``cid``: locations, limits and options."""
    c = dict(CONFIGS[cid])
    g = c["g"]
    n = g * g
    c["id"] = cid
    c["n"] = n
    c["xy"] = grid_xy(g)
    c["a"] = np.full(n, -np.inf)
    c["b"] = upper_limits_uniform(n, 2003 + cid)
    c["seed_shift"] = 11183 + cid
    return c


def random_tlr_factor(n: int, m: int, seed: int, rank_mean: float = 4.0,
                      rank_max: int = 32, zero_frac: float = 0.3,
                      offdiag_scale: float = 0.5):
    """A random lower-triangular factor in tile-low-rank form.

    Returns (diag, ranks, U, V) in the host exchange layout of the library:
    diag is a list of dense lower-triangular m_i x m_i tiles; ranks[i, j]
    (i > j) the rank of tile (i, j); U[(i, j)] is m_i x k, V[(i, j)] is
    m_j x k, and the tile equals U @ V.T.  Rows have norm of order one so
    that the conditional limits stay in the range a spatial factor gives.
    """
    r = (n + m - 1) // m
    sizes = [min(m, n - i * m) for i in range(r)]
    rng_state = seed
    cnt = [0]

    def draw(k):
        out = uniform01(rng_state, k, cnt[0])
        cnt[0] += k
        return out

    diag = []
    for i in range(r):
        mi = sizes[i]
        t = draw(mi * mi).reshape(mi, mi)
        low = np.tril((2.0 * t - 1.0) * 0.5 / math.sqrt(max(mi, 1)), -1)
        d = 0.4 + 0.6 * draw(mi)
        diag.append(low + np.diag(d))
    ranks = np.zeros((r, r), dtype=np.int32)
    for i in range(r):
        for j in range(i):
            u = draw(2)
            if u[0] < zero_frac:
                k = 0
            else:
                k = 1 + int(-math.log(1.0 - u[1]) * max(rank_mean - 1.0, 0.0))
            ranks[i, j] = min(k, rank_max, sizes[i], sizes[j])
    U, V = {}, {}
    for i in range(r):
        kr = int(ranks[i, :i].sum())
        sc = offdiag_scale / math.sqrt(max(kr, 1))
        for j in range(i):
            k = int(ranks[i, j])
            U[(i, j)] = sc * (2.0 * draw(sizes[i] * k).reshape(sizes[i], k) - 1.0) * math.sqrt(3.0)
            V[(i, j)] = (2.0 * draw(sizes[j] * k).reshape(sizes[j], k) - 1.0) * math.sqrt(3.0 / sizes[j])
    return diag, ranks, U, V


def _normals(state: int, count: int, start: int) -> np.ndarray:
    """Box-Muller standard normals from pairs of SplitMix64 uniforms."""
    pairs = (count + 1) // 2
    u = uniform01(state, 2 * pairs, start)
    u1 = 1.0 - u[0::2]          # (0, 1]
    u2 = u[1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * pairs)
    z[0::2] = rad * np.cos(2.0 * math.pi * u2)
    z[1::2] = rad * np.sin(2.0 * math.pi * u2)
    return z[:count]


def serving_stream(count: int = 2000, rate: float = 20.0):
    """Request stream of the serving workload (skew-normal-likelihood shaped).

    Request q draws from SplitMix64 state 20260 + q, in order: grid side g,
    MVN/MVT type, nu, beta, then z (n normals) and delta (n uniforms);
    b_i = delta_i * z_i, a_i = -inf.  Poisson arrival gaps at ``rate`` per
    second come from the separate stream with state 5.
    """
    gaps = -np.log(1.0 - uniform01(5, count)) / rate
    t = np.cumsum(gaps)
    reqs = []
    for q in range(count):
        st = 20260 + q
        u = uniform01(st, 4, 0)
        g = (32, 64, 96, 128)[min(int(4 * u[0]), 3)]
        mvt = bool(u[1] < 0.3)
        nu = (5.0 if u[2] < 0.5 else 10.0) if mvt else 0.0
        beta = 0.05 + 0.25 * u[3]
        n = g * g
        z = _normals(st, n, 4)
        zs = 4 + 2 * ((n + 1) // 2)
        delta = 0.5 + 1.5 * uniform01(st, n, zs)
        reqs.append(dict(q=q, arrival=float(t[q]), g=g, n=n, nu=nu, beta=beta,
                         xy=grid_xy(g), a=np.full(n, -np.inf), b=delta * z,
                         m=128, N=10_000, M=10, seed_shift=11183 + 5 * 100_000 + q))
    return reqs
