"""Outer loop on the GPU likelihood: the library's hcov_fit (Nelder-Mead over
(sigma2, ell, nu) on the H-matrix log-likelihood) against the same simplex
search driven from Python through hcov_nm_minimize with the H-likelihood as
objective (identical evaluation histories), and the objective values it saw
against the dense FP64 likelihood of the oracle."""
import numpy as np
import pytest

import workloads
from oracle import dense
from paper_1709_08625_amd import hcov

pytestmark = pytest.mark.gpu


def test_fit_matches_python_driven_search_and_dense_optimum():
    n, nug, eps, leaf = 1500, 1e-4, 1e-9, 32
    truth = (1.0, 0.1, 1.2)
    locs, xi = workloads.uniform(n, seed=21)
    z = dense.sample_field(locs, xi, *truth, nug)
    theta0 = np.array([1.2, 0.08, 1.32])          # truth x (1.2, 0.8, 1.1)
    steps = [0.01, 0.04, 0.02]
    evals = 40
    # two contexts built the same way: a context keeps the rank hints of its
    # last factorisation (they set the sketch widths of the next one), so two
    # searches agree bit for bit when each starts from a fresh context
    H = hcov.HCov(locs, (*theta0, nug), eps=eps, leaf=leaf, eta=2.0)
    H2 = hcov.HCov(locs, (*theta0, nug), eps=eps, leaf=leaf, eta=2.0)
    try:
        th, ll, ne, hist = H.fit(z, theta0, nug, max_evals=evals, steps=steps)

        def f(x):
            try:
                H2.set_theta((x[0], x[1], x[2], nug))
                return -H2.loglik(z)[0]
            except hcov.HcovError:
                return float("inf")

        th2, f2, ne2, hist2 = hcov.nm_minimize(f, theta0, steps, max_evals=evals)
    finally:
        H.close()
        H2.close()
    assert ne == ne2 == evals
    for (a, fa), (b, fb) in zip(hist, hist2):
        assert np.array_equal(a, b) and fa == fb
    assert np.array_equal(th, th2) and -ll == f2

    # every objective value the search saw is the dense FP64 likelihood to
    # the parity tolerance (checked at the first 8 distinct points)
    import math
    seen = 0
    for x, fx in hist:
        if not np.isfinite(fx) or seen >= 8:
            continue
        ll0, ld0, q0 = dense.loglik_parts(locs, z, x[0], x[1], x[2], nug)
        S = 0.5 * n * math.log(2 * math.pi) + abs(ld0) / 2 + q0 / 2
        assert abs(-fx - ll0) / S < 1e-6
        seen += 1
    assert seen == 8
    # the search improved on its start
    assert -ll < hist[0][1]
