"""Univariate functions the SOV recursion needs (Section 2.1, Eq. 2).

Phi is the standard normal CDF, Phi^-1 its quantile, and chi_nu^-1 the chi
quantile that scales the limits of the Student-t form (Eq. 4, "mvt"
algorithm).  Library routines (scipy.special, Cephes-derived) serve as the
steps; what is written here is how they are combined:

* chi_nu^-1(u) = sqrt(2 * P^-1(nu/2, u)), since S^2/2 ~ Gamma(nu/2) when
  S ~ chi_nu, with P the regularized lower incomplete gamma function.
* the tail of the one-sided case, where Phi(b') underflows the double range,
  goes through log Phi and the quantile of a log-probability.
"""

from __future__ import annotations

import numpy as np
from scipy import special as _sp

# Below this probability a difference of CDFs is handled in the log domain.
TINY = 1e-300


def Phi(x):
    return _sp.ndtr(x)


def log_Phi(x):
    return _sp.log_ndtr(x)


def Phi_inv(u):
    return _sp.ndtri(u)


def Phi_inv_log(log_u):
    """Phi^-1(exp(log_u)) without forming exp(log_u)."""
    return _sp.ndtri_exp(log_u)


def chi_inv(nu: float, u):
    """Quantile of the chi distribution with nu degrees of freedom."""
    return np.sqrt(2.0 * _sp.gammaincinv(0.5 * nu, u))


def phi(x):
    """Standard normal density (zero at +-inf)."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        return np.where(np.isfinite(x), np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi), 0.0)
