"""Dense-oracle parity at n = 32,768 (GPU): the FP64 H path against the
exact FP64 log-likelihood of Eq. (1) for the 128k jittered-grid and the 512k
uniform benchmark parameters at the largest size the dense oracle holds
(fixtures tests/golden/dense32k_*.npz, written by
tests/golden/make_dense32k.py from the oracle alone), within the FP64
tolerance |dL|/S <= 1e-6 for likelihood, log-determinant and quadratic form.
"""
import math
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
N = 32768
CASES = {
    # name: (locations, eps, leaf)
    "cfg2-32k": (lambda: workloads.jitter_grid(N, 182, seed=7)[0], 1e-8, 64),
    "cfg4-32k": (lambda: workloads.uniform(N, seed=N)[0], 1e-7, 128),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_dense32k_parity(name):
    from paper_1709_08625_amd import hcov
    gen, eps, leaf = CASES[name]
    f = np.load(os.path.join(HERE, f"dense32k_{name}.npz"), allow_pickle=False)
    z = f["z"].astype(np.float64)
    th = tuple(float(t) for t in f["theta"])
    ll0, ld0, q0 = float(f["loglik"]), float(f["logdet"]), float(f["quad"])
    locs = gen()
    h = hcov.HCov(locs, th, eps=eps, leaf=leaf, eta=2.0)
    try:
        ll, ld, q = h.loglik(z)
        st = h.stats()
    finally:
        h.close()
    S = 0.5 * N * math.log(2 * math.pi) + abs(ld0) / 2 + q0 / 2
    print(f"{name}: |dL|/S {abs(ll - ll0) / S:.2e} logdet {abs(ld - ld0) / S:.2e} q {abs(q - q0) / S:.2e} "
          f"(retries {st['n_sketch_retries']}, mean rank {st['mean_rank']:.1f})")
    assert abs(ll - ll0) / S < 1e-6
    assert abs(ld - ld0) / S < 1e-6
    assert abs(q - q0) / S < 1e-6
