"""Arbitrary-precision brute-force log-likelihood for tiny n (oracle; test
infrastructure only).

Evaluates Eq. (1) of Sec. 1 with every entry from Eq. (3) at ``dps`` decimal
digits: determinant and C^{-1} Z by mpmath LU.  No Cholesky, no scipy: an
implementation independent of ``oracle.dense`` used to pin it.
"""
import mpmath

from .matern import matern_mp


def loglik_mp(locs, z, sigma2, ell, nu, nugget, dps=50):
    """Return (L, log|C|, Z^T C^{-1} Z) as mpmath numbers."""
    n = len(z)
    with mpmath.workdps(dps):
        C = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                dx = mpmath.mpf(float(locs[i][0])) - mpmath.mpf(float(locs[j][0]))
                dy = mpmath.mpf(float(locs[i][1])) - mpmath.mpf(float(locs[j][1]))
                h = mpmath.sqrt(dx * dx + dy * dy)
                C[i, j] = matern_mp(h, sigma2, ell, nu, dps=dps)
            C[i, i] += mpmath.mpf(nugget)
        zz = mpmath.matrix([mpmath.mpf(float(v)) for v in z])
        det = mpmath.det(C)
        x = mpmath.lu_solve(C, zz)
        quad = sum(zz[i] * x[i] for i in range(n))
        logdet = mpmath.log(det)
        ll = -mpmath.mpf(n) / 2 * mpmath.log(2 * mpmath.pi) - logdet / 2 - quad / 2
        return ll, logdet, quad
