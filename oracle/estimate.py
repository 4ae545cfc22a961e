"""Probability estimate and its standard error from per-sample log P.

Section 2.1 (remark after the MVN algorithm): the mean and the standard
deviation of the integrand over well designed points give the estimate and
its error.  Section 4 (last paragraph): the relative error is the Monte
Carlo standard error over the mean.  Reading taken: randomized QMC with M
independent shifts; the estimate of shift s is the mean over its N points,
the estimate is the mean over shifts and the standard error is the standard
deviation of the M shift means divided by sqrt(M) (one sigma).  Everything
is computed after scaling by exp(-max_s L_s), so log P may be far below the
double range.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import logsumexp


def shift_log_means(logp: np.ndarray) -> np.ndarray:
    """L_s = log(mean_k exp(logp[s, k])) for each shift (row)."""
    N = logp.shape[1]
    with np.errstate(divide="ignore"):
        return logsumexp(logp, axis=1) - math.log(N)


def combine(Ls: np.ndarray) -> dict:
    """Estimate, standard error and relative error from the shift log-means."""
    M = len(Ls)
    mx = float(np.max(Ls))
    if not np.isfinite(mx):
        return dict(log_p=-math.inf, p=0.0, std_err=0.0, rel_err=math.nan, log_p_shift=Ls)
    e = np.exp(Ls - mx)
    mean = float(np.mean(e))
    se = math.sqrt(float(np.sum((e - mean) ** 2)) / (M * (M - 1)))
    log_p = mx + math.log(mean)
    return dict(log_p=log_p, p=math.exp(log_p), std_err=se * math.exp(mx),
                rel_err=se / mean, log_p_shift=Ls)


def estimate(logp: np.ndarray) -> dict:
    return combine(shift_log_means(logp))
