"""Pins of the oracle's setup: covariance, Morton order, truncation, reordering."""

import math

import numpy as np

from oracle import factor as F
from oracle import reorder as R
from oracle import special as sf
import synth


def test_exp_kernel_values():
    xy = np.array([[0.0, 0.0], [1.0, 1.0], [0.3, 0.4]])
    S = F.exp_cov(xy, 0.25)
    assert np.all(np.diag(S) == 1.0)
    assert abs(S[0, 1] - math.exp(-math.sqrt(2.0) / 0.25)) < 1e-16
    assert abs(S[0, 2] - math.exp(-0.5 / 0.25)) < 1e-16
    assert np.array_equal(S, S.T)


def test_morton_order_of_a_4x4_grid():
    # Z-order with the first coordinate's bits in the more significant place.
    perm = F.morton_order(synth.grid_xy(4))
    assert perm.tolist() == [0, 1, 4, 5, 2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15]


def test_morton_blocks_are_compact():
    # On a 2^k grid every aligned block of 4^j consecutive positions is a square.
    g = 16
    xy = synth.grid_xy(g)
    perm = F.morton_order(xy)
    for blk in range(0, g * g, 16):
        pts = np.round(xy[perm[blk:blk + 16]] * (g - 1)).astype(int)
        assert np.ptp(pts[:, 0]) == 3 and np.ptp(pts[:, 1]) == 3


def test_truncation_bounds_each_tile():
    n, m, tol = 128, 32, 1e-5
    xy = synth.grid_xy(int(math.isqrt(n)))
    perm = F.morton_order(xy)
    L = np.linalg.cholesky(F.exp_cov(xy, 0.1, perm))
    diag, ranks, U, V, hits = F.tlr_from_dense(L, m, tol)
    assert hits == 0
    for i in range(n // m):
        assert np.array_equal(diag[i], np.tril(L[i * m:(i + 1) * m, i * m:(i + 1) * m]))
        for j in range(i):
            T = L[i * m:(i + 1) * m, j * m:(j + 1) * m]
            E = T - U[(i, j)] @ V[(i, j)].T
            assert np.linalg.norm(E, 2) <= tol * (1 + 1e-9)
            assert ranks[i, j] <= m
    exact = F.tlr_from_dense(L, m, 0.0)[:4]
    assert np.allclose(F.TLRRows(*exact).dense(), L, atol=1e-13)


def test_rank_cap_counts_hits():
    n, m = 64, 16
    xy = synth.grid_xy(8)
    L = np.linalg.cholesky(F.exp_cov(xy, 0.5))
    _, ranks, _, _, hits = F.tlr_from_dense(L, m, 1e-12, cap=2)
    assert ranks.max() <= 2 and hits > 0


def test_univariate_conditioning_independent_case():
    # Sigma diagonal: conditioning changes nothing, so the order sorts the
    # interval probabilities and the score is their exact product.
    rng = np.random.default_rng(0)
    m = 12
    sd = rng.uniform(0.5, 2, m)
    a = np.where(rng.random(m) < 0.5, -np.inf, rng.uniform(-2, 0, m))
    b = rng.uniform(0.1, 3, m)
    order, lp = R.univariate_conditioning(np.diag(sd ** 2), a, b)
    probs = np.array([0.5 * math.erfc(-b[i] / sd[i] / math.sqrt(2)) -
                      (0.0 if a[i] == -np.inf else 0.5 * math.erfc(-a[i] / sd[i] / math.sqrt(2)))
                      for i in range(m)])
    assert order.tolist() == np.argsort(probs, kind="stable").tolist()
    assert abs(lp - np.sum(np.log(probs))) < 1e-12


def test_univariate_conditioning_bivariate_by_hand():
    # Two variables: pick the smaller marginal probability, then condition the
    # other on the truncated mean of the first (computed here from scratch).
    rho = 0.6
    S = np.array([[1.0, rho], [rho, 1.0]])
    a = np.array([-np.inf, -np.inf])
    b = np.array([1.5, 0.2])
    order, lp = R.univariate_conditioning(S, a, b)
    assert order.tolist() == [1, 0]
    p1 = 0.5 * math.erfc(-0.2 / math.sqrt(2))
    ybar = -math.exp(-0.02) / math.sqrt(2 * math.pi) / p1   # E[Z | Z < 0.2]
    b2 = (1.5 - rho * ybar) / math.sqrt(1 - rho * rho)
    p2 = 0.5 * math.erfc(-b2 / math.sqrt(2))
    assert abs(lp - math.log(p1 * p2)) < 1e-13


def test_block_reorder_sorts_blocks_and_keeps_them_whole():
    g, m = 16, 16
    xy = synth.grid_xy(g)
    n = g * g
    base = F.morton_order(xy)
    S = F.exp_cov(xy, 0.1)
    b = synth.upper_limits_uniform(n, 7)
    a = np.full(n, -np.inf)
    perm = R.block_reorder(S, a, b, m, base)
    assert sorted(perm.tolist()) == list(range(n))
    scores = []
    for q in range(n // m):
        blk = perm[q * m:(q + 1) * m]
        assert set(blk.tolist()) in [set(base[t * m:(t + 1) * m].tolist()) for t in range(n // m)]
        order, lp = R.univariate_conditioning(S[np.ix_(blk, blk)], a[blk], b[blk])
        assert order.tolist() == list(range(m))     # within-block order is the chosen one
        scores.append(lp)
    assert all(scores[q] <= scores[q + 1] + 1e-12 for q in range(len(scores) - 1))


def test_block_reorder_constant_problem_keeps_order():
    # Constant correlation and equal limits: every block scores the same, so
    # the reordering has nothing to do (the paper's Section 4 remark).
    n, m = 24, 6
    S = 0.4 * np.ones((n, n)) + 0.6 * np.eye(n)
    base = np.arange(n)
    perm = R.block_reorder(S, np.full(n, -np.inf), np.full(n, 0.5), m, base)
    assert perm.tolist() == list(range(n))


def test_phi_density():
    assert abs(sf.phi(0.0) - 1 / math.sqrt(2 * math.pi)) < 1e-17
    assert sf.phi(np.inf) == 0.0 and sf.phi(-np.inf) == 0.0


# ---------------------------------------------- iterative block reordering

def _random_spd(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n))
    return X @ X.T / n + 0.5 * np.eye(n)


def test_iterative_reorder_factor_is_cholesky_of_reordered_covariance():
    g, m = 12, 16
    xy = synth.grid_xy(g)
    n = g * g
    S = F.exp_cov(xy, 0.2)
    base = F.morton_order(xy)
    b = synth.upper_limits_uniform(n, 21)
    a = np.full(n, -np.inf)
    perm, L = R.iterative_block_reorder(S, a, b, m, base)
    assert sorted(perm.tolist()) == list(range(n))
    assert np.allclose(L, np.tril(L))
    assert np.all(np.diag(L) > 0)
    P = S[np.ix_(perm, perm)]
    assert np.abs(L @ L.T - P).max() < 1e-12
    # the blocks stay whole (the ragged last one stays last)
    blocks = [set(base[t:t + m].tolist()) for t in range(0, n, m)]
    for q in range(0, n, m):
        assert set(perm[q:q + m].tolist()) in blocks
    assert set(perm[(n // m) * m:].tolist()) == set(base[(n // m) * m:].tolist())


def test_iterative_reorder_of_independent_blocks_is_block_reorder():
    # With no correlation between blocks, conditioning changes neither the
    # blocks' covariances nor their limits, so every step sees the first
    # step's scores: the result is the plain block reordering.
    m, r = 5, 6
    n = m * r
    S = np.zeros((n, n))
    for q in range(r):
        S[q * m:(q + 1) * m, q * m:(q + 1) * m] = _random_spd(m, 100 + q)
    rng = np.random.default_rng(3)
    b = rng.uniform(-0.5, 2.5, n)
    a = b - rng.uniform(0.5, 3.0, n)
    base = np.arange(n)
    perm, L = R.iterative_block_reorder(S, a, b, m, base)
    assert perm.tolist() == R.block_reorder(S, a, b, m, base).tolist()


def test_iterative_reorder_single_block_is_univariate_conditioning():
    n = 9
    S = _random_spd(n, 7)
    rng = np.random.default_rng(8)
    b = rng.uniform(-1, 2, n)
    a = np.full(n, -np.inf)
    perm, L = R.iterative_block_reorder(S, a, b, n, np.arange(n))
    order, _ = R.univariate_conditioning(S, a, b)
    assert perm.tolist() == order.tolist()
    assert np.abs(L - np.linalg.cholesky(S[np.ix_(order, order)])).max() < 1e-13


def test_iterative_reorder_second_step_scores_the_conditional_problem():
    # After the first block is chosen, the remaining blocks must be scored on
    # the Gaussian conditional distribution given that block at its
    # truncated mean mu = L_11 y (original coordinates): covariance
    # S22 - S21 S11^-1 S12 and limits shifted by S21 S11^-1 mu.
    m = 4
    n = 3 * m
    S = _random_spd(n, 11)
    rng = np.random.default_rng(12)
    b = rng.uniform(-0.5, 1.5, n)
    a = np.full(n, -np.inf)
    base = np.arange(n)
    perm, L = R.iterative_block_reorder(S, a, b, m, base)
    first = perm[:m]
    # the first block is the plain block reordering's first choice, in its order
    assert first.tolist() == R.block_reorder(S, a, b, m, base)[:m].tolist()
    order, _, y = R.univariate_conditioning(S[np.ix_(first, first)], a[first], b[first], with_means=True)
    assert order.tolist() == list(range(m))
    S11 = S[np.ix_(first, first)]
    mu = np.linalg.cholesky(S11) @ y
    rest = np.array([i for i in base if i not in set(first.tolist())])
    S21 = S[np.ix_(rest, first)]
    C = S[np.ix_(rest, rest)] - S21 @ np.linalg.solve(S11, S21.T)
    shift = S21 @ np.linalg.solve(S11, mu)
    ac, bc = a[rest] - shift, b[rest] - shift
    # score the two remaining blocks of the conditional problem
    lps = []
    for q in range(2):
        sl = slice(q * m, (q + 1) * m)
        lps.append(R.univariate_conditioning(C[sl, sl], ac[sl], bc[sl])[1])
    winner = rest[int(np.argmin(lps)) * m:(int(np.argmin(lps)) + 1) * m]
    assert set(perm[m:2 * m].tolist()) == set(winner.tolist())
    assert np.abs(L @ L.T - S[np.ix_(perm, perm)]).max() < 1e-12
