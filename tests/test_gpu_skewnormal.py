"""GPU parity of the skew-normal likelihood client (Section 5, Eq. 6).

The library computes the density term, the limits c and the covariance
Gamma on the device, factors Gamma into TLR form and estimates the MVN
probability term.  Against the oracle: the density term and c from the
dense formulas, the factor against the Cholesky factor of the oracle's Gamma
in the same order (truncated tile by tile), and the probability term against
the oracle's estimator on the exported factor with the same limits.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import factor as OF
from oracle import reorder as OR
from oracle import skewnormal as SN

pytestmark = pytest.mark.gpu

PARAMS = dict(xi=0.2, sigma1=1.0, beta1=0.3, sigma2=1.0, beta2=0.3)


@pytest.fixture(scope="module")
def T():
    from paper_2003_11183_amd import tlrqmc
    return tlrqmc


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def observations(g, seed):
    """Locations on a g x g grid with unit distance 1/15 (Section 5.2) and a
    draw z = xi 1 + A x + B |y| of the model with PARAMS."""
    xy = synth.grid_xy(g) * ((g - 1) / 15.0)
    n = g * g
    x = synth.workloads._normals(700 + seed, n, 0)
    y = synth.workloads._normals(800 + seed, n, 0)
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    K1 = PARAMS["sigma1"] ** 2 * np.exp(-d / PARAMS["beta1"])
    B = PARAMS["sigma2"] ** 2 * np.exp(-d / PARAMS["beta2"])
    z = PARAMS["xi"] + np.linalg.cholesky(K1) @ x + B @ np.abs(y)
    return xy, z


@pytest.mark.parametrize("order", [0, 2])
def test_skewnormal_loglik_against_oracle(T, ctx, order):
    g, m, tol, N, M, seed = 20, 64, 1e-5, 500, 4, 41
    xy, z = observations(g, 1)
    n = g * g
    res = T.skewnormal_loglik(ctx, xy, z, N=N, M=M, seed=seed, m=m, tol=tol, order=order, return_factor=True,
                              **PARAMS)
    log_phi, c, Gamma = SN.terms(xy, z, **PARAMS)
    assert abs(res["log_density"] - log_phi) <= 1e-10 * abs(log_phi)
    assert np.abs(res["c"] - c).max() <= 1e-9 * max(1.0, np.abs(c).max())
    F = res["factor"]
    perm, diag, ranks, U, V = F.export()
    base = OF.morton_order(xy)
    if order == 0:
        assert perm.tolist() == base.tolist()
        L = np.linalg.cholesky(Gamma[np.ix_(perm, perm)])
    else:
        ref_perm, L = OR.iterative_block_reorder(Gamma, np.full(n, -np.inf), c, m, base)
        assert perm.tolist() == ref_perm.tolist()
    for i in range(len(diag)):
        assert np.abs(np.tril(diag[i]) - L[i * m:(i + 1) * m, i * m:(i + 1) * m]).max() <= 1e-9
        for j in range(i):
            T_ = L[i * m:(i + 1) * m, j * m:(j + 1) * m]
            assert np.linalg.norm(T_ - U[(i, j)] @ V[(i, j)].T, 2) <= tol * 1.01 + 1e-9
    # probability term: the oracle's estimator on the exported factor, same limits
    cl = res["c"]
    ref, _ = oracle.probability((diag, ranks, U, V), np.full(n, -np.inf), cl[perm], 0.0, N, M, seed)
    assert abs(res["log_prob"] - ref["log_p"]) <= 1e-10 * max(1.0, abs(ref["log_p"]))
    total = n * math.log(2.0) + res["log_density"] + res["log_prob"]
    assert abs(res["loglik"] - total) <= 1e-12 * abs(total)
    F.free()


def test_skewnormal_without_skewness_is_gaussian(T, ctx):
    # sigma2 = 0: B = 0, Gamma = I and c = 0, so the probability term is 2^-n
    # and the log-likelihood is the Gaussian log-density.
    xy, z = observations(12, 2)
    n = len(z)
    p = dict(PARAMS, sigma2=0.0)
    res = T.skewnormal_loglik(ctx, xy, z, N=200, M=4, seed=3, m=48, **p)
    assert np.abs(res["c"]).max() == 0.0
    assert abs(res["log_prob"] + n * math.log(2.0)) <= 1e-10 * n
    log_phi, _, _ = SN.terms(xy, z, **p)
    assert abs(res["loglik"] - log_phi) <= 1e-9 * abs(log_phi)
