"""Pins of the oracle's estimator against closed forms and quadrature.

Each pin fixes the result by mathematics that does not go through the
oracle's code: exact products of univariate CDFs (zero-variance cases),
the equicorrelated orthant probability 1/(n+1), one-dimensional quadrature
representations, Plackett's bivariate formula and the Student-t CDF.  The
mutation tests at the end plant plausible mistakes in the oracle and check
that some pin catches each of them.
"""

import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from oracle import factor as F
from oracle import sov

INF = math.inf


def _phi_diff(a, b):
    """Phi(b) - Phi(a) from libm erfc, taking the accurate tail."""
    if a > 0:
        return 0.5 * math.erfc(a / math.sqrt(2)) - 0.5 * math.erfc(b / math.sqrt(2))
    return 0.5 * math.erfc(-b / math.sqrt(2)) - 0.5 * math.erfc(-a / math.sqrt(2))


def _within(res, exact, k=3.0):
    return abs(res["p"] - exact) <= k * res["std_err"] + 1e-15


def _equicorr(n, rho):
    return (1 - rho) * np.eye(n) + rho * np.ones((n, n))


# --------------------------------------------------------------- exact cases

@pytest.mark.parametrize("a,b", [(-INF, 1.3), (-0.5, 2.0), (0.7, 3.1), (2.5, INF),
                                 (-INF, -3.0), (5.0, 6.0), (-2.0, -1.0)])
def test_univariate_every_sample_exact(a, b):
    L = np.array([[1.0]])
    lp = oracle.sample_logp(L, [a], [b], 0.0, 5, 4, 1, np.arange(1, 300))
    assert np.allclose(lp, math.log(_phi_diff(a, b)), rtol=1e-14, atol=1e-15)


def test_univariate_deep_tail_log_space():
    # Phi(-40) underflows the double range; log Phi from the Mills series.
    x = -40.0
    series = (-x * x / 2 - math.log(-x) - 0.5 * math.log(2 * math.pi)
              + math.log(1 - 1 / x ** 2 + 3 / x ** 4 - 15 / x ** 6 + 105 / x ** 8))
    lp = oracle.sample_logp(np.array([[1.0]]), [-INF], [x], 0.0, 5, 4, 0, np.arange(1, 50))
    assert np.allclose(lp, series, rtol=1e-12)


def diag_case_ok(n=40, seed=3):
    rng = np.random.default_rng(seed)
    sd = rng.uniform(0.5, 2.0, n)
    a = np.where(rng.random(n) < 0.5, -INF, rng.uniform(-2, 1.5, n))
    b = np.where(np.isinf(a), rng.uniform(-1, 3, n), a + rng.uniform(0.1, 2, n))
    L = np.diag(sd)
    lp = oracle.sample_logp(L, a, b, 0.0, 17, 3, 2, np.arange(1, 200))
    want = sum(math.log(_phi_diff(a[i] / sd[i], b[i] / sd[i])) for i in range(n))
    return np.allclose(lp, want, rtol=1e-13, atol=0)


def test_independent_limits_every_sample_is_the_product():
    assert diag_case_ok()


# ------------------------------------------------------------ orthant 1/(n+1)

def orthant_ok(n, N=2000, M=16, seed=11, tlr_m=0):
    L = np.linalg.cholesky(_equicorr(n, 0.5))
    fac = L if tlr_m == 0 else F.tlr_from_dense(L, tlr_m, 1e-13)[:4]
    res, _ = oracle.probability(fac, np.full(n, -INF), np.zeros(n), 0.0, N, M, seed)
    return _within(res, 1.0 / (n + 1))


@pytest.mark.parametrize("n", [3, 10, 40])
def test_equicorrelated_orthant(n):
    assert orthant_ok(n)


def test_equicorrelated_orthant_tlr_rank_one_tiles():
    n, m = 48, 8
    L = np.linalg.cholesky(_equicorr(n, 0.5))
    diag, ranks, U, V, _ = F.tlr_from_dense(L, m, 1e-12)
    assert np.all(ranks[np.tril_indices(n // m, -1)] == 1)
    assert orthant_ok(n, tlr_m=m)


def equicorr_quadrature_ok(n=12, rho=0.3, seed=4):
    rng = np.random.default_rng(seed)
    b = rng.uniform(-0.5, 2.5, n)
    c, s = math.sqrt(rho), math.sqrt(1 - rho)
    exact = integrate.quad(lambda z: stats.norm.pdf(z) * np.prod(stats.norm.cdf((b - c * z) / s)),
                           -12, 12, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
    L = np.linalg.cholesky(_equicorr(n, rho))
    res, _ = oracle.probability(L, np.full(n, -INF), b, 0.0, 4000, 16, 21)
    return _within(res, exact)


def test_equicorrelated_arbitrary_limits_quadrature():
    assert equicorr_quadrature_ok()


# ------------------------------------------------------------------ bivariate

def _plackett(b1, b2, rho):
    """Phi_2(-inf, b; rho) = Phi(b1)Phi(b2) + (2pi)^-1 int_0^rho exp(...)/sqrt(1-r^2) dr."""
    f = lambda r: math.exp(-(b1 * b1 - 2 * r * b1 * b2 + b2 * b2) / (2 * (1 - r * r))) / math.sqrt(1 - r * r)
    return stats.norm.cdf(b1) * stats.norm.cdf(b2) + integrate.quad(f, 0, rho, epsabs=1e-15)[0] / (2 * math.pi)


def _box2(a, b, rho):
    """P(a < X < b) for the standard bivariate normal, by inclusion-exclusion."""
    def F2(x1, x2):
        if x1 == -INF or x2 == -INF:
            return 0.0
        if x1 == INF:
            return stats.norm.cdf(x2)
        if x2 == INF:
            return stats.norm.cdf(x1)
        return _plackett(x1, x2, rho)
    return F2(b[0], b[1]) - F2(a[0], b[1]) - F2(b[0], a[1]) + F2(a[0], a[1])


def bivariate_ok(a, b, rho, N=3000, M=16, seed=8):
    L = np.linalg.cholesky(np.array([[1.0, rho], [rho, 1.0]]))
    res, _ = oracle.probability(L, np.array(a, float), np.array(b, float), 0.0, N, M, seed)
    return _within(res, _box2(a, b, rho))


@pytest.mark.parametrize("a,b,rho", [((-INF, -INF), (0.3, -0.4), 0.6),
                                     ((-1.0, 0.2), (1.5, 2.0), -0.5),
                                     ((0.4, -INF), (2.0, 1.0), 0.8),
                                     ((0.5, 0.6), (INF, 3.0), 0.3)])
def test_bivariate_plackett(a, b, rho):
    assert bivariate_ok(a, b, rho)


def test_block_diagonal_is_product_of_blocks():
    rhos = [0.7, -0.3, 0.5]
    bs = [(0.2, 1.1), (1.4, -0.2), (0.0, 0.9)]
    L = np.zeros((6, 6))
    b = np.zeros(6)
    exact = 1.0
    for q, (rho, bb) in enumerate(zip(rhos, bs)):
        L[2 * q:2 * q + 2, 2 * q:2 * q + 2] = np.linalg.cholesky(np.array([[1, rho], [rho, 1.0]]))
        b[2 * q:2 * q + 2] = bb
        exact *= _plackett(bb[0], bb[1], rho)
    fac = F.tlr_from_dense(L, 2, 1e-14)[:4]       # all off-diagonal tiles rank 0
    res, _ = oracle.probability(fac, np.full(6, -INF), b, 0.0, 4000, 16, 3)
    assert _within(res, exact)


# ----------------------------------------------------------------- Student-t

def t_univariate_ok(nu, t, N=4000, M=16, seed=5):
    res, _ = oracle.probability(np.array([[1.0]]), np.array([-INF]), np.array([t]), nu, N, M, seed)
    if nu == 1:
        exact = 0.5 + math.atan(t) / math.pi
    elif nu == 2:
        exact = 0.5 + t / (2 * math.sqrt(t * t + 2))
    else:
        exact = stats.t.cdf(t, nu)
    return _within(res, exact)


@pytest.mark.parametrize("nu,t", [(1, 0.8), (2, -0.6), (5, 1.7), (7, -1.1), (10, 2.3)])
def test_student_t_univariate_cdf(nu, t):
    assert t_univariate_ok(nu, t)


def test_student_t_identity_scale_quadrature():
    n, nu = 5, 7.0
    b = np.array([0.5, 1.2, -0.3, 2.0, 0.9])
    f = lambda s: stats.chi.pdf(s, nu) * np.prod(stats.norm.cdf(s * b / math.sqrt(nu)))
    exact = integrate.quad(f, 0, 30, epsabs=1e-14, limit=200)[0]
    res, _ = oracle.probability(np.eye(n), np.full(n, -INF), b, nu, 4000, 16, 9)
    assert _within(res, exact)


def test_student_t_large_nu_tends_to_normal():
    n = 20
    S = F.exp_cov(np.random.default_rng(1).random((n, 2)), 0.3)
    L = np.linalg.cholesky(S)
    b = np.linspace(0.2, 2.5, n)
    ks = np.arange(1, 100)
    lpn = oracle.sample_logp(L, np.full(n, -INF), b, 0.0, 12, 2, 0, ks)
    lpt = oracle.sample_logp(L, np.full(n, -INF), b, 1e12, 12, 2, 0, ks)
    # chi_nu / sqrt(nu) = 1 + O(nu^-1/2): 1e-6 at nu = 1e12
    assert np.allclose(lpt, lpn, rtol=2e-5)


# -------------------------------------------------------- structure and error

def test_tlr_exact_tiles_match_dense_per_sample():
    n, m = 96, 16
    xy = np.random.default_rng(2).random((n, 2))
    L = np.linalg.cholesky(F.exp_cov(xy, 0.2) + 1e-10 * np.eye(n))
    fac = F.tlr_from_dense(L, m, 0.0)[:4]
    b = np.random.default_rng(3).uniform(0, 3, n)
    ks = np.arange(1, 64)
    l1 = oracle.sample_logp(L, np.full(n, -INF), b, 0.0, 4, 2, 1, ks)
    l2 = oracle.sample_logp(fac, np.full(n, -INF), b, 0.0, 4, 2, 1, ks)
    assert np.allclose(l1, l2, rtol=1e-12)


def test_reordering_leaves_the_estimate_within_error():
    n = 30
    rng = np.random.default_rng(6)
    xy = rng.random((n, 2))
    S = F.exp_cov(xy, 0.2)
    b = rng.uniform(0.0, 2.5, n)
    perm = rng.permutation(n)
    r1, _ = oracle.probability(np.linalg.cholesky(S), np.full(n, -INF), b, 0.0, 4000, 16, 1)
    Sp = S[np.ix_(perm, perm)]
    r2, _ = oracle.probability(np.linalg.cholesky(Sp), np.full(n, -INF), b[perm], 0.0, 4000, 16, 2)
    assert abs(r1["p"] - r2["p"]) <= 3 * math.hypot(r1["std_err"], r2["std_err"])


def coverage_ok(seeds=range(24), n=5):
    z = []
    for sd in seeds:
        L = np.linalg.cholesky(_equicorr(n, 0.5))
        res, _ = oracle.probability(L, np.full(n, -INF), np.zeros(n), 0.0, 64, 10, 1000 + sd)
        z.append((res["p"] - 1.0 / (n + 1)) / res["std_err"])
    z = np.array(z)
    rms = float(np.sqrt(np.mean(z ** 2)))
    return np.mean(np.abs(z) < 2.5) >= 0.8 and 0.4 < rms < 2.0


def test_standard_error_has_the_right_scale():
    # (P_hat - P) / SE over independent seeds behaves like N(0, 1) (t_9).
    assert coverage_ok()


# ------------------------------------------------------- planted mistakes

def test_planted_mistakes_are_caught(monkeypatch):
    orig = sov._step

    # 1. drop the d_i term of the quantile argument (the listing's typo)
    def no_d(ah, bh, w):
        ld, y = orig(ah, bh, w)
        lower = ah <= 0
        from oracle import special as sf
        e = sf.Phi(bh)
        d = sf.Phi(ah)
        y2 = sf.Phi_inv(np.clip(w * (e - d), 1e-300, 1 - 1e-16))
        return ld, np.where(lower, y2, y)
    monkeypatch.setattr(sov, "_step", no_d)
    assert not bivariate_ok((-1.0, 0.2), (1.5, 2.0), -0.5)
    monkeypatch.setattr(sov, "_step", orig)

    # 2. wrong sign of y in the complement branch
    def bad_sign(ah, bh, w):
        ld, y = orig(ah, bh, w)
        return ld, np.where(ah > 0, -y, y)
    monkeypatch.setattr(sov, "_step", bad_sign)
    assert not bivariate_ok((0.4, -INF), (2.0, 1.0), 0.8)
    monkeypatch.setattr(sov, "_step", orig)

    # 3. transposed factor (upper triangle read as the row product)
    class Transposed(sov.DenseRows):
        def rows(self, i0, i1):
            return self.L.T[i0:i1, :i1]
    n = 10
    L = np.linalg.cholesky(_equicorr(n, 0.5))
    res, _ = oracle.probability(Transposed(L), np.full(n, -INF), np.zeros(n), 0.0, 2000, 16, 11)
    assert not _within(res, 1.0 / (n + 1))

    # 4. Student-t without the chi scaling of the limits
    import oracle.api as api
    real_chi = api.sf.chi_inv
    monkeypatch.setattr(api.sf, "chi_inv", lambda nu, u: np.full_like(u, math.sqrt(nu)))
    assert not t_univariate_ok(5, 1.7)
    monkeypatch.setattr(api.sf, "chi_inv", real_chi)
