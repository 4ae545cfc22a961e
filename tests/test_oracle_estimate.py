"""Exact pins of the oracle's estimate and standard error (oracle/estimate.py).

Section 2.1 (remark after the MVN algorithm): the estimate and its error are
the mean and the standard deviation of the integrand's values; Section 4
(last paragraph): relative error = standard error / mean.  With M randomly
shifted lattices the estimate is the mean of the M shift means and its
standard error the sample standard deviation of those means over sqrt(M):

    SE = sqrt( sum_s (P_s - P)^2 / (M (M - 1)) ).

The values below are worked by hand from that definition, so a wrong
denominator (M^2, i.e. the population variance, or M (M + 1)), a missing
square root or a log-space slip changes them; the planted variants at the
end must fail the same checks.
"""

import math

import numpy as np
import pytest

from oracle import estimate as est

LOG = np.log


def _combine_pins_hold(combine) -> bool:
    """The hand-worked cases, each a few lines of arithmetic."""
    ok = True
    # P_s = 1, 2, 3: mean 2; squared deviations 1 + 0 + 1 = 2; 2 / (3 * 2) = 1/3.
    r = combine(LOG(np.array([1.0, 2.0, 3.0])))
    ok &= math.isclose(r["log_p"], math.log(2.0), rel_tol=0, abs_tol=1e-15)
    ok &= math.isclose(r["p"], 2.0, rel_tol=1e-15)
    ok &= math.isclose(r["std_err"], math.sqrt(1.0 / 3.0), rel_tol=1e-14)
    ok &= math.isclose(r["rel_err"], math.sqrt(1.0 / 3.0) / 2.0, rel_tol=1e-14)
    # M = 2: SE = |P_1 - P_2| / 2 exactly (deviations +-1, 2 / (2 * 1) = 1).
    r = combine(LOG(np.array([1.0, 3.0])))
    ok &= math.isclose(r["std_err"], 1.0, rel_tol=1e-14)
    # P_s = 2, 4, 6, 8: mean 5; deviations 9 + 1 + 1 + 9 = 20; 20 / (4 * 3) = 5/3.
    r = combine(LOG(np.array([2.0, 4.0, 6.0, 8.0])))
    ok &= math.isclose(r["p"], 5.0, rel_tol=1e-15)
    ok &= math.isclose(r["std_err"], math.sqrt(5.0 / 3.0), rel_tol=1e-14)
    # equal shift means: zero error
    r = combine(LOG(np.array([0.25, 0.25, 0.25])))
    ok &= r["std_err"] == 0.0 and math.isclose(r["p"], 0.25, rel_tol=1e-15)
    # far below the double range: P_s = 1, 2, 3 times e^-2000 (only logs exist)
    r = combine(LOG(np.array([1.0, 2.0, 3.0])) - 2000.0)
    ok &= math.isclose(r["log_p"], math.log(2.0) - 2000.0, rel_tol=1e-15)
    ok &= r["p"] == 0.0 and r["std_err"] == 0.0
    ok &= math.isclose(r["rel_err"], math.sqrt(1.0 / 3.0) / 2.0, rel_tol=1e-12)
    return bool(ok)


def test_combine_matches_hand_worked_values():
    assert _combine_pins_hold(est.combine)


def test_combine_all_shifts_dead():
    r = est.combine(np.array([-np.inf, -np.inf]))
    assert r["log_p"] == -np.inf and r["p"] == 0.0 and r["std_err"] == 0.0 and math.isnan(r["rel_err"])


def test_combine_one_dead_shift():
    # P_s = 0, 2: mean 1, deviations 1 + 1 = 2, 2 / (2 * 1) = 1
    with np.errstate(divide="ignore"):
        r = est.combine(LOG(np.array([0.0, 2.0])))
    assert math.isclose(r["p"], 1.0, rel_tol=1e-15)
    assert math.isclose(r["std_err"], 1.0, rel_tol=1e-14)


def test_shift_log_means_hand_values():
    # shift 0: P = 1, 3 -> mean 2; shift 1: P = 2, 2 -> 2; shift 2: P = 0, 4 -> 2
    with np.errstate(divide="ignore"):
        lp = LOG(np.array([[1.0, 3.0], [2.0, 2.0], [0.0, 4.0]]))
    Ls = est.shift_log_means(lp)
    assert np.allclose(Ls, math.log(2.0), rtol=0, atol=1e-15)
    # deep underflow of every sample: log-sum-exp keeps the value
    Ls = est.shift_log_means(LOG(np.array([[1.0, 3.0]])) - 5000.0)
    assert math.isclose(Ls[0], math.log(2.0) - 5000.0, rel_tol=1e-15)


def test_estimate_over_samples_and_shifts():
    # per-sample P (2 shifts x 3 samples): shift means 2 and 4 -> P = 3,
    # SE = |2 - 4| / 2 = 1
    lp = LOG(np.array([[1.0, 2.0, 3.0], [4.0, 4.0, 4.0]]))
    r = est.estimate(lp)
    assert math.isclose(r["p"], 3.0, rel_tol=1e-15)
    assert math.isclose(r["std_err"], 1.0, rel_tol=1e-14)


# ------------------------------------------------------- planted mistakes

def _variant(denominator):
    """combine() with the variance denominator replaced: the plausible slips."""
    def combine(Ls):
        M = len(Ls)
        mx = float(np.max(Ls))
        e = np.exp(Ls - mx)
        mean = float(np.mean(e))
        se = math.sqrt(float(np.sum((e - mean) ** 2)) / denominator(M))
        log_p = mx + math.log(mean)
        return dict(log_p=log_p, p=math.exp(log_p), std_err=se * math.exp(mx), rel_err=se / mean)
    return combine


@pytest.mark.parametrize("name,den", [
    ("population variance, M^2", lambda M: M * M),
    ("M (M + 1)", lambda M: M * (M + 1)),
    ("no 1/M (standard deviation, not error)", lambda M: M - 1),
])
def test_planted_denominators_fail_the_pins(name, den):
    assert not _combine_pins_hold(_variant(den)), name


def test_right_denominator_passes_through_the_same_harness():
    # the harness itself accepts the definition when written out again
    assert _combine_pins_hold(_variant(lambda M: M * (M - 1)))
