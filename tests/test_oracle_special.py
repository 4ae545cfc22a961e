"""Pins of the oracle's univariate functions: closed forms and libm."""

import math

import numpy as np

from oracle import special as sf


def test_phi_known_values():
    assert sf.Phi(0.0) == 0.5
    assert abs(sf.Phi_inv(0.975) - 1.959963984540054) < 1e-15
    assert abs(sf.Phi(1.959963984540054) - 0.975) < 1e-16


def test_phi_against_libm_erfc():
    xs = np.linspace(-37.0, 8.0, 4001)
    ref = np.array([0.5 * math.erfc(-x / math.sqrt(2.0)) for x in xs])
    got = sf.Phi(xs)
    # Condition number of Phi at x is about 1 + x^2 in the lower tail (the
    # argument -x/sqrt2 is itself rounded), so the bound scales with it.
    assert np.all(np.abs(got - ref) <= 4e-16 * (1.0 + xs * xs) * ref + 1e-300)


def test_phi_symmetry_and_roundtrip():
    xs = np.linspace(-37.0, 8.0, 901)
    assert np.allclose(sf.Phi(xs) + sf.Phi(-xs), 1.0, rtol=0, atol=2e-16)
    back = sf.Phi_inv(sf.Phi(xs))
    # A rounding of Phi(x) by one ulp moves the quantile by ulp / phi(x).
    tol = 4e-16 * np.maximum(sf.Phi(xs), 1e-300) / sf.phi(xs) + 1e-14 * np.abs(xs)
    assert np.all(np.abs(back - xs) <= tol)


def test_log_phi_and_log_quantile():
    xs = np.linspace(-30.0, 5.0, 351)
    ref = np.array([math.log(0.5 * math.erfc(-x / math.sqrt(2.0))) for x in xs])
    assert np.allclose(sf.log_Phi(xs), ref, rtol=1e-14, atol=1e-15)
    # Deep tail: Mills-ratio series log Phi(x) = -x^2/2 - log(-x) - log(2 pi)/2
    # + log(1 - 1/x^2 + 3/x^4 - 15/x^6 + ...), x = -100.
    x = -100.0
    series = (-x * x / 2 - math.log(-x) - 0.5 * math.log(2 * math.pi)
              + math.log(1 - 1 / x ** 2 + 3 / x ** 4 - 15 / x ** 6))
    assert abs(sf.log_Phi(x) - series) < 1e-12 * abs(series)
    lus = np.array([-1e-3, -0.7, -5.0, -50.0, -700.0, -5000.0])
    ys = sf.Phi_inv_log(lus)
    assert np.allclose(sf.log_Phi(ys), lus, rtol=1e-13, atol=1e-16)
    mid = lus > -700
    assert np.allclose(ys[mid], sf.Phi_inv(np.exp(lus[mid])), rtol=1e-13)


def test_chi_inverse_closed_forms():
    us = np.array([1e-12, 1e-6, 0.01, 0.3, 0.5, 0.77, 0.99, 1 - 1e-9])
    # nu = 2: S^2/2 ~ Exp(1), so chi_2^-1(u) = sqrt(-2 log(1 - u))
    assert np.allclose(sf.chi_inv(2.0, us), np.sqrt(-2.0 * np.log1p(-us)), rtol=1e-13)
    # nu = 1: S = |Z|, P(|Z| <= x) = 2 Phi(x) - 1
    ref1 = np.array([_half_normal_quantile(u) for u in us])
    got1 = sf.chi_inv(1.0, us)
    assert np.allclose(got1, ref1, rtol=1e-11)
    # nu = 3: F(x) = erf(x/sqrt2) - sqrt(2/pi) x exp(-x^2/2)
    x3 = sf.chi_inv(3.0, us)
    F3 = np.array([math.erf(x / math.sqrt(2)) - math.sqrt(2 / math.pi) * x * math.exp(-x * x / 2)
                   for x in x3])
    assert np.allclose(F3, us, rtol=1e-10, atol=1e-16)


def _half_normal_quantile(u):
    """x >= 0 with erf(x / sqrt 2) = u, by bisection on libm erf / erfc."""
    lo, hi = 0.0, 40.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        below = (math.erf(mid / math.sqrt(2.0)) < u) if u < 0.5 else \
                (math.erfc(mid / math.sqrt(2.0)) > 1.0 - u)
        if below:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
