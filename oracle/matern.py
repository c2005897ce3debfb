"""Matérn covariance, Eq. (3) of Sec. 2.1 (oracle; test infrastructure only).

    C(h; theta) = sigma^2 / (2^(nu-1) Gamma(nu)) * (h/ell)^nu * K_nu(h/ell)

with theta = (ell, nu, sigma^2), ell, nu, sigma^2 > 0 and K_nu the modified
Bessel function of the second kind.  The argument is h/ell exactly as printed
(no sqrt(2 nu) factor).  C(0) = sigma^2 is the h -> 0 limit, since
x^nu K_nu(x) -> 2^(nu-1) Gamma(nu).

K_nu comes from ``scipy.special.kv`` (a library routine serving as one step);
it is pinned separately against ``mpmath.besselk`` at 50 digits.
"""
import math

import numpy as np
from scipy import special


def matern(h, sigma2, ell, nu):
    """Eq. (3) evaluated elementwise on distances ``h`` (array, h >= 0)."""
    h = np.asarray(h, dtype=np.float64)
    x = h / ell
    out = np.empty_like(x)
    zero = x == 0.0
    out[zero] = sigma2
    xs = x[~zero]
    norm = sigma2 / (2.0 ** (nu - 1.0) * math.gamma(nu))
    out[~zero] = norm * xs ** nu * special.kv(nu, xs)
    # kv underflows to 0 for very large x; the product is then 0 as well.
    out[~zero] = np.where(np.isfinite(out[~zero]), out[~zero], 0.0)
    return out


def matern_half_integer(h, sigma2, ell, nu):
    """Closed forms of Eq. (3) for nu in {1/2, 3/2, 5/2} (Sec. 2.1 names nu=1/2
    as the exponential kernel); x = h/ell.

    nu=1/2: sigma^2 exp(-x); nu=3/2: sigma^2 (1+x) exp(-x);
    nu=5/2: sigma^2 (1 + x + x^2/3) exp(-x).
    These follow from K_{n+1/2} being elementary (DLMF 10.47.9, 10.49.12).
    """
    x = np.asarray(h, dtype=np.float64) / ell
    e = np.exp(-x)
    if nu == 0.5:
        return sigma2 * e
    if nu == 1.5:
        return sigma2 * (1.0 + x) * e
    if nu == 2.5:
        return sigma2 * (1.0 + x + x * x / 3.0) * e
    raise ValueError("closed form only for nu in {0.5, 1.5, 2.5}")


def besselk_mp(nu, x, dps=50):
    """K_nu(x) at ``dps`` decimal digits by mpmath: an implementation
    independent of scipy's, used only to pin ``scipy.special.kv``."""
    import mpmath

    with mpmath.workdps(dps):
        return mpmath.besselk(mpmath.mpf(nu), mpmath.mpf(x))


def matern_mp(h, sigma2, ell, nu, dps=50):
    """Eq. (3) at ``dps`` digits (mpmath), scalar ``h``."""
    import mpmath

    with mpmath.workdps(dps):
        if h == 0:
            return mpmath.mpf(sigma2)
        x = mpmath.mpf(h) / mpmath.mpf(ell)
        nu_ = mpmath.mpf(nu)
        return (mpmath.mpf(sigma2) / (2 ** (nu_ - 1) * mpmath.gamma(nu_))
                * x ** nu_ * mpmath.besselk(nu_, x))
