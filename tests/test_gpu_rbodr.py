"""GPU parity of the block reordering during the Cholesky factorization.

The library's tlr_factor_rbodr (device Cholesky steps, host scoring) against
the oracle's dense form of the same algorithm on the same covariance and
limits: the order must be identical, the factor equal up to the tile
truncation, and the estimate on the library's factor must match the oracle
on the exported factor at the FP64 bar.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import factor as OF
from oracle import reorder as OR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2003_11183_amd import tlrqmc
    return tlrqmc


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def check_factor(F, L, m, tol):
    perm, diag, ranks, U, V = F.export()
    n = L.shape[0]
    r = len(diag)
    for i in range(r):
        i0, i1 = i * m, min((i + 1) * m, n)
        assert np.abs(np.tril(diag[i]) - L[i0:i1, i0:i1]).max() <= 1e-11
        for j in range(i):
            T_ = L[i0:i1, j * m:(j + 1) * m]
            assert np.linalg.norm(T_ - U[(i, j)] @ V[(i, j)].T, 2) <= tol * 1.01 + 1e-12
    return perm, (diag, ranks, U, V)


def run_case(T, ctx, cov, S, base, a, b, m, tol, seed=5):
    n = len(a)
    F = T.Factor.build_reordered(ctx, cov, a, b, m, tol)
    perm_ref, L = OR.iterative_block_reorder(S, a, b, m, base)
    assert F.perm.tolist() == perm_ref.tolist()
    perm, fac = check_factor(F, L, m, tol)
    assert perm.tolist() == perm_ref.tolist()
    # the estimate on the library's factor, against the oracle on the same factor
    res = T.probability(ctx, F, a, b, 400, 4, seed, return_logp=True)
    ref, ref_logp = oracle.probability(fac, a[perm], b[perm], 0.0, 400, 4, seed)
    fin = np.isfinite(ref_logp)
    err = np.abs(res["logp"][fin] - ref_logp[fin]) / np.maximum(1.0, np.abs(ref_logp[fin]))
    assert err.max() <= 1e-10
    assert abs(res["log_p"] - ref["log_p"]) <= 1e-10 * max(1.0, abs(ref["log_p"]))
    return F


def test_rbodr_grid_upper_limits(T, ctx):
    g, m, beta, tol = 32, 64, 0.1, 1e-5
    xy = synth.grid_xy(g)
    n = g * g
    S = OF.exp_cov(xy, beta)
    b = synth.upper_limits_uniform(n, 31)
    a = np.full(n, -np.inf)
    F = run_case(T, ctx, {"xy": xy, "beta": beta}, S, OF.morton_order(xy), a, b, m, tol)
    assert F.perm.tolist() != OF.morton_order(xy).tolist()


def test_rbodr_ragged_two_sided(T, ctx):
    g, m, beta, tol = 30, 64, 0.2, 1e-5
    xy = synth.grid_xy(g)
    n = g * g
    S = OF.exp_cov(xy, beta)
    b = synth.upper_limits_uniform(n, 32, hi=3.0)
    a = b - 2.5
    run_case(T, ctx, {"xy": xy, "beta": beta}, S, OF.morton_order(xy), a, b, m, tol)


def test_rbodr_dense_sigma(T, ctx):
    n, m = 300, 32
    rng = np.random.default_rng(9)
    X = rng.standard_normal((n, n))
    S = X @ X.T / n + 0.3 * np.eye(n)
    b = rng.uniform(-0.5, 2.0, n)
    a = b - rng.uniform(1.0, 3.0, n)
    run_case(T, ctx, {"sigma": S}, S, np.arange(n), a, b, m, 1e-5)
