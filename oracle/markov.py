"""Exact O(n) log-likelihoods of Matérn fields observed along a line (oracle;
test infrastructure only).

For points s_i = (x_i, y0) on a horizontal line the Matérn field of Eq. (3)
restricted to the line is a stationary Gauss-Markov process in x, so Eq. (1)
is available exactly without any n x n matrix:

* nu = 1/2 (the exponential kernel named in Sec. 2.1) is an AR(1) chain:
  with x sorted, rho_i = exp(-(x_{i+1} - x_i)/ell) and no nugget,
      log|C| = n log sigma^2 + sum_i log(1 - rho_i^2),
      Z^T C^{-1} Z = Z_1^2/sigma^2
                     + sum_i (Z_{i+1} - rho_i Z_i)^2 / (sigma^2 (1 - rho_i^2)).
* with a nugget, or for nu = 3/2, the Kalman filter on the state-space form
  (Hartikainen & Särkkä 2010) gives the exact likelihood through the
  prediction-error decomposition.

Points are sorted by x internally (ties are not allowed); Z follows its points.
"""
import math

import numpy as np


def _sorted(x, z):
    order = np.argsort(x, kind="stable")
    xs = np.asarray(x, dtype=np.float64)[order]
    if np.any(np.diff(xs) <= 0):
        raise ValueError("points on the line must be distinct")
    return xs, np.asarray(z, dtype=np.float64)[order]


def ou_loglik(x, z, sigma2, ell):
    """Closed-form AR(1) log-likelihood (nu = 1/2, nugget 0).
    Returns (L, logdet, quad)."""
    xs, zs = _sorted(x, z)
    n = len(xs)
    rho = np.exp(-np.diff(xs) / ell)
    one_m = 1.0 - rho * rho
    logdet = n * math.log(sigma2) + float(np.sum(np.log(one_m)))
    quad = zs[0] ** 2 / sigma2 + float(np.sum((zs[1:] - rho * zs[:-1]) ** 2 / (sigma2 * one_m)))
    ll = -0.5 * n * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * quad
    return ll, logdet, quad


def _kalman(xs, zs, F_of, Q_of, P0, H, r):
    """Prediction-error decomposition: returns (L, logdet, quad) with
    logdet = sum log S_i and quad = sum e_i^2 / S_i."""
    m = P0.shape[0]
    mean = np.zeros(m)
    P = P0.copy()
    logdet = 0.0
    quad = 0.0
    for i in range(len(xs)):
        if i > 0:
            d = xs[i] - xs[i - 1]
            F = F_of(d)
            mean = F @ mean
            P = F @ P @ F.T + Q_of(d, F)
        S = float(H @ P @ H) + r
        e = zs[i] - float(H @ mean)
        K = (P @ H) / S
        mean = mean + K * e
        P = P - np.outer(K, H @ P)
        logdet += math.log(S)
        quad += e * e / S
    n = len(xs)
    ll = -0.5 * n * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * quad
    return ll, logdet, quad


def kalman_loglik(x, z, sigma2, ell, nu, nugget):
    """Exact log-likelihood for nu in {1/2, 3/2} with nugget tau^2 >= 0.

    nu = 1/2: scalar state, F = exp(-d/ell), stationary variance sigma^2.
    nu = 3/2 with C(h) = sigma^2 (1 + h/ell) exp(-h/ell), lam = 1/ell: state
    (f, f'), F(d) = exp(-lam d) [[1 + lam d, d], [-lam^2 d, 1 - lam d]],
    stationary covariance diag(sigma^2, lam^2 sigma^2), Q = Pinf - F Pinf F^T.
    """
    xs, zs = _sorted(x, z)
    if nu == 0.5:
        P0 = np.array([[sigma2]])
        H = np.array([1.0])
        F_of = lambda d: np.array([[math.exp(-d / ell)]])
        Q_of = lambda d, F: P0 - F @ P0 @ F.T
    elif nu == 1.5:
        lam = 1.0 / ell
        P0 = np.diag([sigma2, lam * lam * sigma2])
        H = np.array([1.0, 0.0])

        def F_of(d):
            e = math.exp(-lam * d)
            return e * np.array([[1 + lam * d, d], [-lam * lam * d, 1 - lam * d]])

        Q_of = lambda d, F: P0 - F @ P0 @ F.T
    else:
        raise ValueError("state-space form implemented for nu in {0.5, 1.5}")
    return _kalman(xs, zs, F_of, Q_of, P0, H, float(nugget))
