"""The allocation-free Matérn evaluation (GPU, collected last): hcov_matern_eval_noalloc
against hcov_matern_eval, which stages through hipMalloc'd buffers; both run
the same device kernel, so the outputs agree bit for bit.  Two calls in a
row, the second smaller, then an oversized request (rejected)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NOALLOC_MAX = 262144


def _call(L, fn, theta, h):
    from paper_1709_08625_amd import hcov
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.full_like(h, np.nan)
    dp = C.POINTER(C.c_double)
    rc = getattr(L, fn)(hcov._theta(theta), h.ctypes.data_as(dp), out.ctypes.data_as(dp), C.c_int64(h.size))
    return rc, out


def test_noalloc_matches_allocating_entry_point():
    from paper_1709_08625_amd import hcov
    L = hcov.lib()
    L.hcov_matern_eval_noalloc.argtypes = [hcov.Theta, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64]
    rng = np.random.default_rng(11)
    # first call: the largest size, a generic nu (K_nu series and quadrature)
    h1 = rng.uniform(0.0, 2.0, NOALLOC_MAX)
    th1 = (1.3, 0.1, 0.8, 1e-4)
    rc, a1 = _call(L, "hcov_matern_eval_noalloc", th1, h1)
    assert rc == hcov.OK
    rc, b1 = _call(L, "hcov_matern_eval", th1, h1)
    assert rc == hcov.OK
    assert np.array_equal(a1, b1)
    # second call, smaller, another theta: the staging keeps the first call's
    # tail, which must not leak into the result
    h2 = rng.uniform(0.0, 1.0, 1000)
    th2 = (0.7, 0.05, 1.5, 0.0)
    rc, a2 = _call(L, "hcov_matern_eval_noalloc", th2, h2)
    assert rc == hcov.OK
    rc, b2 = _call(L, "hcov_matern_eval", th2, h2)
    assert np.array_equal(a2, b2)
    assert np.all(np.isfinite(a2))
    # beyond the fixed staging: rejected before any device work
    rc, _ = _call(L, "hcov_matern_eval_noalloc", th1, np.zeros(NOALLOC_MAX + 1))
    assert rc == hcov.EINVAL
