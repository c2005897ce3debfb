"""The benchmark's own configuration at full size (marked gpu).

n = 512,000 uniform points (seed 0), theta = (1, 0.08, 0.8, 1e-4), leaf 128,
eta 2, eps 1e-7 -- the workload `bench.py` times.  The dense oracle cannot
hold this matrix (2.1 TB), so the checks are on sampled outputs the oracle
computes one by one and on properties that hold at any size:

* rows of H x against the exact rows of C x (Eq. (3) Matérn entries from the
  oracle, one row of n entries at a time), relative to sum_j |C_ij x_j|;
* the stand-alone forward solve gives the same quadratic form as the sweep
  with the fused right-hand side, bit for bit, and a second evaluation at
  the same theta repeats the likelihood bit for bit.
"""
import numpy as np
import pytest

import workloads
from oracle import matern

pytestmark = pytest.mark.gpu

N = 512000
THETA = (1.0, 0.08, 0.8, 1e-4)


def test_full_size_matvec_rows_and_sweep_properties():
    from paper_1709_08625_amd import hcov
    locs, _ = workloads.uniform(N, seed=0)
    h = hcov.HCov(locs, THETA, eps=1e-7, leaf=128, eta=2.0)
    try:
        x = np.random.default_rng(11).standard_normal(N)
        y = h.matvec(x)
        rows = np.random.default_rng(12).choice(N, 8, replace=False)
        worst = 0.0
        for i in rows:
            d = np.hypot(locs[:, 0] - locs[i, 0], locs[:, 1] - locs[i, 1])
            c = matern.matern(d, THETA[0], THETA[1], THETA[2])
            c[i] += THETA[3]
            ref = float(c @ x)
            scale = float(np.abs(c) @ np.abs(x))
            worst = max(worst, abs(float(y[i]) - ref) / scale)
        print(f"n={N}: worst sampled row |Hx - Cx| / sum|C x| = {worst:.2e}")
        assert worst < 1e-6
        z = np.random.default_rng(13).standard_normal(N)
        ll, ld, q = h.loglik(z)
        assert np.isfinite(ll) and np.isfinite(ld) and q > 0.0
        _, qf = h.forward(z)
        assert qf == q
        h.set_theta(THETA)
        assert h.loglik(z) == (ll, ld, q)
    finally:
        h.close()
