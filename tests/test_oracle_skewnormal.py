"""Pins of the oracle's skew-normal likelihood (Section 5, Eq. 5-6)."""

import math

import numpy as np
from scipy import integrate
from scipy.special import log_ndtr, ndtr

from oracle import skewnormal as SN


def exact_log_mvn_independent(c, Gamma):
    """Phi_n(-inf, c; Gamma) for a diagonal Gamma: a product of Phi."""
    assert np.allclose(Gamma, np.diag(np.diag(Gamma)), atol=1e-14)
    return float(log_ndtr(c / np.sqrt(np.diag(Gamma))).sum())


def bivariate_cdf(h, k, rho):
    """Phi_2((-inf, -inf), (h, k); [[1, rho], [rho, 1]]) by one integral:
    int_{-inf}^{h} phi(x) Phi((k - rho x) / sqrt(1 - rho^2)) dx."""
    s = math.sqrt(1.0 - rho * rho)
    f = lambda x: math.exp(-0.5 * x * x) / math.sqrt(2 * math.pi) * ndtr((k - rho * x) / s)
    v, _ = integrate.quad(f, -np.inf, h, epsabs=1e-14, epsrel=1e-12)
    return v


def log_mvn_2(c, Gamma):
    sd = np.sqrt(np.diag(Gamma))
    rho = Gamma[0, 1] / (sd[0] * sd[1])
    return math.log(bivariate_cdf(c[0] / sd[0], c[1] / sd[1], rho))


def test_univariate_is_azzalini_skew_normal():
    # n = 1: Z = xi + a X + b |Y| has density 2 phi(z - xi; a^2 + b^2)
    # Phi(b (z - xi) / (a sqrt(a^2 + b^2))) (Azzalini's skew-normal).
    xy = np.array([[0.3, 0.7]])
    s1, s2, xi = 0.8, 1.1, 0.25
    a, b = s1, s2 ** 2
    for z in (-2.0, -0.3, 0.0, 0.9, 3.1):
        got = SN.loglik(xy, [z], xi, s1, 0.3, s2, 0.2, exact_log_mvn_independent)
        w2 = a * a + b * b
        ref = (math.log(2) - 0.5 * math.log(2 * math.pi * w2) - (z - xi) ** 2 / (2 * w2)
               + float(log_ndtr(b * (z - xi) / (a * math.sqrt(w2)))))
        assert abs(got - ref) < 1e-13


def test_far_apart_locations_factorise():
    # Correlations exp(-d / beta) vanish: the log-likelihood is the sum of the
    # univariate ones.
    xy = np.array([[0.0, 0.0], [50.0, 0.0], [0.0, 50.0], [50.0, 50.0]])
    z = np.array([0.4, -1.2, 2.0, 0.1])
    s1, b1, s2, b2, xi = 1.3, 0.2, 0.7, 0.1, -0.1
    got = SN.loglik(xy, z, xi, s1, b1, s2, b2, exact_log_mvn_independent)
    ref = sum(SN.loglik(xy[i:i + 1], z[i:i + 1], xi, s1, b1, s2, b2, exact_log_mvn_independent) for i in range(4))
    assert abs(got - ref) < 1e-12


def test_univariate_density_integrates_to_one_and_has_the_model_mean():
    xy = np.array([[0.0, 0.0]])
    s1, s2, xi = 0.6, 0.9, 0.3
    f = lambda z: math.exp(SN.loglik(xy, [z], xi, s1, 0.3, s2, 0.3, exact_log_mvn_independent))
    tot, _ = integrate.quad(f, -np.inf, np.inf, epsabs=1e-13)
    mean, _ = integrate.quad(lambda z: z * f(z), -np.inf, np.inf, epsabs=1e-13)
    assert abs(tot - 1.0) < 1e-9
    # E Z = xi + B E|Y| = xi + sigma2^2 sqrt(2 / pi)
    assert abs(mean - (xi + s2 ** 2 * math.sqrt(2 / math.pi))) < 1e-8


def test_bivariate_density_integrates_to_one_and_has_the_model_mean():
    # Two correlated locations: the density of Eq. 6 (with its bivariate
    # normal CDF by quadrature) is a probability density whose mean is
    # xi 1 + B E|Y| = xi 1 + B 1 sqrt(2 / pi).
    xy = np.array([[0.0, 0.0], [0.15, 0.1]])
    s1, b1, s2, b2, xi = 0.9, 0.4, 0.8, 0.25, 0.1

    def dens(z1, z2):
        return math.exp(SN.loglik(xy, [z1, z2], xi, s1, b1, s2, b2, log_mvn_2))

    lo, hi = -7.0, 9.0
    tot, _ = integrate.dblquad(lambda z2, z1: dens(z1, z2), lo, hi, lo, hi, epsabs=1e-10, epsrel=1e-10)
    m1, _ = integrate.dblquad(lambda z2, z1: z1 * dens(z1, z2), lo, hi, lo, hi, epsabs=1e-10, epsrel=1e-10)
    assert abs(tot - 1.0) < 1e-7
    B = SN.kernel(xy, s2 ** 2, b2)
    assert abs(m1 - (xi + B[0].sum() * math.sqrt(2 / math.pi))) < 1e-6
