"""Dense FP64 Gaussian log-likelihood (oracle; test infrastructure only).

Eq. (1), Sec. 1:
    L(theta) = -n/2 log(2 pi) - 1/2 log|C(theta)| - 1/2 Z^T C(theta)^{-1} Z,
with C_ij = C(||s_i - s_j||; theta) from Eq. (3) and the nugget tau^2 added to
the diagonal only (C := C + tau^2 I, Sec. 4 and Sec. 5.2).

Through the exact Cholesky factor C = L L^T this is Eq. (2) with the exact
factor in place of the H-approximation:
    log|C| = 2 sum_i log L_ii,   Z^T C^{-1} Z = v^T v  with  L v = Z.

Two factorisations are provided: an own unblocked right-looking Cholesky
(column by column, for n up to a few thousand) and LAPACK ``dpotrf`` via scipy;
each pins the other.
"""
import math

import numpy as np
from scipy import linalg

from .matern import matern


def distances(locs):
    """Euclidean distance matrix ||s_i - s_j|| of 2-D locations (n x 2)."""
    locs = np.asarray(locs, dtype=np.float64)
    dx = locs[:, 0][:, None] - locs[:, 0][None, :]
    dy = locs[:, 1][:, None] - locs[:, 1][None, :]
    return np.sqrt(dx * dx + dy * dy)


def cov_block(locs_a, locs_b, sigma2, ell, nu):
    """Block C(||a_i - b_j||) of Eq. (3) between two location sets (no
    nugget): the entries of cov_matrix for rows a and columns b, for
    assembling large dense matrices a block of rows at a time."""
    a = np.asarray(locs_a, dtype=np.float64)
    b = np.asarray(locs_b, dtype=np.float64)
    dx = a[:, 0][:, None] - b[:, 0][None, :]
    dy = a[:, 1][:, None] - b[:, 1][None, :]
    return matern(np.sqrt(dx * dx + dy * dy), sigma2, ell, nu)


def cov_matrix(locs, sigma2, ell, nu, nugget):
    """Dense C(theta) + tau^2 I (Eq. (3) entries; nugget on the diagonal)."""
    C = matern(distances(locs), sigma2, ell, nu)
    C[np.diag_indices_from(C)] += nugget
    return C


def cholesky_unblocked(C):
    """Own lower Cholesky C = L L^T, one column at a time (textbook
    right-looking form).  Raises ValueError on a non-positive pivot."""
    A = np.array(C, dtype=np.float64, copy=True)
    n = A.shape[0]
    L = np.zeros_like(A)
    for j in range(n):
        d = A[j, j]
        if not d > 0.0:
            raise ValueError(f"matrix not SPD: pivot {j} = {d}")
        ljj = math.sqrt(d)
        L[j, j] = ljj
        col = A[j + 1:, j] / ljj
        L[j + 1:, j] = col
        # Schur complement update of the trailing block (lower part suffices,
        # the full update keeps the code plain).
        A[j + 1:, j + 1:] -= np.outer(col, col)
    return L


def cholesky_lapack(C):
    """Lower Cholesky by LAPACK dpotrf (scipy)."""
    return linalg.cholesky(np.asarray(C, dtype=np.float64), lower=True)


def cholesky_torch(C):
    """Lower Cholesky by LAPACK dpotrf through PyTorch's CPU backend (MKL).
    The same factorisation as cholesky_lapack; used for n >= 32768, where the
    OpenBLAS build behind NumPy/SciPy in this environment fails."""
    import torch
    return torch.linalg.cholesky(torch.from_numpy(np.ascontiguousarray(C, dtype=np.float64))).numpy()


def forward_solve_torch(L, z):
    """Solve L v = z by LAPACK triangular solve through PyTorch (MKL)."""
    import torch
    Lt = torch.from_numpy(np.ascontiguousarray(L, dtype=np.float64))
    zt = torch.from_numpy(np.ascontiguousarray(z, dtype=np.float64)).reshape(-1, 1)
    return torch.linalg.solve_triangular(Lt, zt, upper=False).reshape(-1).numpy()


def forward_solve_unblocked(L, z):
    """Solve L v = z by plain forward substitution."""
    n = L.shape[0]
    v = np.zeros(n)
    for i in range(n):
        v[i] = (z[i] - L[i, :i] @ v[:i]) / L[i, i]
    return v


def forward_solve_lapack(L, z):
    """Solve L v = z by LAPACK dtrtrs (scipy)."""
    return linalg.solve_triangular(L, z, lower=True)


def logdet_from_factor(L):
    """log|C| = 2 sum log L_ii (Eq. (2))."""
    return 2.0 * float(np.sum(np.log(np.diag(L))))


def loglik_parts(locs, z, sigma2, ell, nu, nugget, own=False):
    """Return (L, logdet, quad) of Eq. (1) via the exact Cholesky factor.

    ``own=True`` uses the unblocked Cholesky and substitution (small n)."""
    C = cov_matrix(locs, sigma2, ell, nu, nugget)
    if own:
        L = cholesky_unblocked(C)
        v = forward_solve_unblocked(L, np.asarray(z, dtype=np.float64))
    else:
        L = cholesky_lapack(C)
        v = forward_solve_lapack(L, np.asarray(z, dtype=np.float64))
    logdet = logdet_from_factor(L)
    quad = float(v @ v)
    n = len(z)
    ll = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * quad
    return ll, logdet, quad


def loglik(locs, z, sigma2, ell, nu, nugget, own=False):
    """Exact log-likelihood of Eq. (1) (returned with the paper's sign, +L)."""
    return loglik_parts(locs, z, sigma2, ell, nu, nugget, own=own)[0]


def solve(locs, z, sigma2, ell, nu, nugget):
    """x = C^{-1} z through the exact factor (forward then backward solve)."""
    C = cov_matrix(locs, sigma2, ell, nu, nugget)
    L = cholesky_lapack(C)
    v = linalg.solve_triangular(L, z, lower=True)
    return linalg.solve_triangular(L.T, v, lower=False)


def sample_field(locs, xi, sigma2, ell, nu, nugget):
    """Z = L xi with the exact factor (the synthetic-data recipe of Sec. 5.1,
    with the dense factor in place of the H-factor)."""
    C = cov_matrix(locs, sigma2, ell, nu, nugget)
    return cholesky_lapack(C) @ np.asarray(xi, dtype=np.float64)
