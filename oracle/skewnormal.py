"""Skew-normal log-likelihood (Section 5, the stochastic generator Eq. 5 and its
density Eq. 6) — test infrastructure, plain dense numpy in FP64.

Model: Z = xi 1 + A X + B |Y| with X, Y independent standard normal vectors;
A is the lower Cholesky factor of sigma1^2 exp(-|h|/beta1) and B the
covariance matrix sigma2^2 exp(-|h|/beta2) on the n locations (Section 5.2).
Density (Eq. 6):

    2^n phi_n(z - xi 1; A A^T + B B^T) Phi_n(-inf, c; Gamma),
    C = A^-1 B,  Gamma = (I + C^T C)^-1,  c = Gamma C^T A^-1 (z - xi 1).

The deterministic terms are written out here; the MVN probability term is
whatever estimator the caller supplies (the oracle's SOV estimator, or an
exact value in the pins).
"""

from __future__ import annotations

import math

import numpy as np


def kernel(xy: np.ndarray, variance: float, beta: float) -> np.ndarray:
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    return variance * np.exp(-d / beta)


def terms(xy, z, xi, sigma1, beta1, sigma2, beta2):
    """Returns (log_phi, c, Gamma): the log-density term, the upper limits
    and the covariance of the MVN probability term of Eq. 6."""
    xy = np.asarray(xy, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = len(z)
    K1 = kernel(xy, sigma1 ** 2, beta1)
    B = kernel(xy, sigma2 ** 2, beta2)
    A = np.linalg.cholesky(K1)
    r = z - xi
    Om = K1 + B @ B.T
    Lo = np.linalg.cholesky(Om)
    u = np.linalg.solve(Lo, r)
    log_phi = -0.5 * (n * math.log(2 * math.pi) + 2 * np.log(np.diag(Lo)).sum() + u @ u)
    C = np.linalg.solve(A, B)
    G = np.eye(n) + C.T @ C
    Gamma = np.linalg.inv(G)
    Gamma = 0.5 * (Gamma + Gamma.T)
    c = Gamma @ (C.T @ np.linalg.solve(A, r))
    return log_phi, c, Gamma


def loglik(xy, z, xi, sigma1, beta1, sigma2, beta2, log_mvn):
    """Eq. 6 in log form; log_mvn(c, Gamma) supplies log Phi_n(-inf, c; Gamma)."""
    log_phi, c, Gamma = terms(xy, z, xi, sigma1, beta1, sigma2, beta2)
    return len(c) * math.log(2.0) + log_phi + log_mvn(c, Gamma)
