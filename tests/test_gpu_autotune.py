"""Empirical choice between the two GEMM kernels (opts.autotune, marked gpu).

The tuned context times every sweep launch both kernels may run and keeps
the faster one; the results differ from the untuned context's by rounding
only (the kernels add a tile's products in different orders), match the
dense oracle to the FP64 tolerance, and repeat bit for bit once tuned.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import dense

pytestmark = pytest.mark.gpu


def test_autotuned_context_matches_untuned_and_oracle():
    from paper_1709_08625_amd import hcov
    n, th = 6000, (1.0, 0.08, 0.8, 1e-4)
    locs, xi = workloads.uniform(n, seed=3)
    z = dense.sample_field(locs, xi, *th)
    out = {}
    for tune in (0, 1):
        H = hcov.HCov(locs, th, eps=1e-9, leaf=64, eta=2.0, opts={"autotune": tune})
        try:
            first = H.loglik(z)
            H.set_theta(th)
            H.profile_begin("gemm")
            again = H.loglik(z)
            _, _, pflops, pbytes = H.profile_end()
            st = H.stats()
            # the planned GEMM work of a factorisation in the stats is what
            # the profiled factorisation's launches add up to
            assert st["gemm_flops_factor"] == pytest.approx(pflops, rel=1e-12) and pflops > 0
            assert st["gemm_bytes_factor"] == pytest.approx(pbytes, rel=1e-12)
        finally:
            H.close()
        out[tune] = (first, again, st)
    ll0, ld0, q0 = dense.loglik_parts(locs, z, *th)
    S = 0.5 * n * math.log(2 * math.pi) + abs(ld0) / 2 + q0 / 2
    (f0, a0, s0), (f1, a1, s1) = out[0], out[1]
    assert s0["n_autotune_switched"] == 0 and s0["n_gemm_grouped"] > 0
    assert a0 == f0 and a1 == f1                # repeats bit for bit
    for a, b in zip(f0, f1):
        assert abs(a - b) / S < 1e-12           # rounding-level differences only
    assert abs(f1[0] - ll0) / S < 1e-6
    print(f"switched {s1['n_autotune_switched']} of the sweep's GEMM launches; "
          f"grouped launches {s0['n_gemm_grouped']} -> {s1['n_gemm_grouped']}")
