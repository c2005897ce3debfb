"""Saturated randomised sketches in the factorisation's recompression (GPU).

A low-rank target of the H-Cholesky sweep is recompressed to accuracy eps
(Sec. 2.2, the same eps for the factor as for C~, Table 5) from a randomised
sketch whose width is a rank estimate plus an oversampling.  When the kept
rank fills the sketch (kept >= width - 1 while the sketch is narrower than the
block) the block's accuracy is not guaranteed: the library doubles that
block's rank hint and redoes the factorisation, or reports HCOV_ERANK.  These
tests force saturation with the smallest oversampling (2) and compare with the
dense FP64 oracle at the stated tolerance |dL|/S <= 1e-6
(S = n/2 log 2 pi + |log|C||/2 + q/2).
"""
import math

import numpy as np
import pytest

import workloads
from oracle import dense

pytestmark = pytest.mark.gpu


def _hc():
    from paper_1709_08625_amd import hcov
    return hcov


def scale(n, ld, q):
    return 0.5 * n * math.log(2 * math.pi) + abs(ld) / 2 + q / 2


CASES = [
    # n, theta, eps, leaf: the uniform nu = 0.8 shape of the 512k benchmark and
    # the nu = 1.5 jittered-grid shape
    (4000, "uniform", (1.0, 0.08, 0.8, 1e-4), 1e-7, 128),
    (3000, "grid", (1.0, 0.05, 1.5, 1e-5), 1e-8, 64),
]


def _inputs(kind, n):
    if kind == "uniform":
        return workloads.uniform(n, seed=21)
    return workloads.jitter_grid(n, int(math.ceil(math.sqrt(n))) + 1, seed=22)


@pytest.mark.parametrize("n,kind,th,eps,leaf", CASES)
def test_forced_saturation_retries_and_matches_dense(n, kind, th, eps, leaf):
    hcov = _hc()
    locs, xi = _inputs(kind, n)
    z = dense.sample_field(locs, xi, *th)
    ll0, ld0, q0 = dense.loglik_parts(locs, z, *th)
    S = scale(n, ld0, q0)
    h = hcov.HCov(locs, th, eps=eps, leaf=leaf, eta=2.0, opts={"oversample": 2})
    ll, ld, q = h.loglik(z)
    st = h.stats()
    print(f"n={n} {kind}: retries={st['n_sketch_retries']} saturated_last={st['sketch_saturated']} "
          f"width={st['mean_sketch_width']:.1f} mean rank {st['mean_rank']:.1f} "
          f"rel ll {abs(ll - ll0) / S:.2e} ld {abs(ld - ld0) / S:.2e} q {abs(q - q0) / S:.2e}")
    assert 1 <= st["n_sketch_retries"] <= 4
    assert st["sketch_saturated"] == 0          # the accepted factorisation had none
    assert abs(ll - ll0) / S < 1e-6
    assert abs(ld - ld0) / S < 1e-6
    assert abs(q - q0) / S < 1e-6
    # a new theta starts from the rank hints the last factorisation left
    r1 = st["n_sketch_retries"]
    th2 = (th[0] * 1.05, th[1] * 0.95, th[2] * 1.03, th[3])
    ll1, ld1, q1 = dense.loglik_parts(locs, z, *th2)
    h.set_theta(th2)
    ll2, _, _ = h.loglik(z)
    st2 = h.stats()
    print(f"  second theta: retries {st2['n_sketch_retries'] - r1} width {st2['mean_sketch_width']:.1f}")
    assert st2["sketch_saturated"] == 0
    assert abs(ll2 - ll1) / scale(n, ld1, q1) < 1e-6
    h.close()


def test_saturation_error_policy():
    hcov = _hc()
    n, kind, th, eps, leaf = CASES[0]
    locs, xi = _inputs(kind, n)
    h = hcov.HCov(locs, th, eps=eps, leaf=leaf, eta=2.0,
                  opts={"oversample": 2, "on_saturation": hcov.SAT_ERROR})
    with pytest.raises(hcov.HcovError) as e:
        h.loglik(xi)
    assert e.value.code == hcov.ERANK
    assert h.stats()["sketch_saturated"] > 0
    # and the factor is not marked as done
    with pytest.raises(hcov.HcovError) as e:
        h.logdet()
    assert e.value.code == hcov.ESTATE
    h.close()


def test_default_oversampling_reports_saturation_state():
    # with the default oversampling: the state is reported, and a second
    # evaluation at a nearby theta starts from the learned rank hints
    hcov = _hc()
    n, kind, th, eps, leaf = CASES[0]
    locs, xi = _inputs(kind, n)
    z = dense.sample_field(locs, xi, *th)
    ll0, ld0, q0 = dense.loglik_parts(locs, z, *th)
    h = hcov.HCov(locs, th, eps=eps, leaf=leaf, eta=2.0)
    ll, ld, q = h.loglik(z)
    st = h.stats()
    print(f"default oversample: retries={st['n_sketch_retries']} width={st['mean_sketch_width']:.1f}")
    assert st["sketch_saturated"] == 0
    assert abs(ll - ll0) / scale(n, ld0, q0) < 1e-6
    h.set_theta((1.05, 0.084, 0.82, 1e-4))
    h.loglik(z)
    st2 = h.stats()
    print(f"  nearby theta: retries {st2['n_sketch_retries'] - st['n_sketch_retries']}")
    assert st2["sketch_saturated"] == 0
    h.close()


def test_sketch_seed():
    # opts.seed draws another Gaussian test matrix: the sketches differ, the
    # likelihood stays within the FP64 tolerance of the dense oracle, and one
    # seed repeats bit for bit
    hcov = _hc()
    n, th = 3000, (1.0, 0.08, 0.8, 1e-4)
    locs, xi = workloads.uniform(n, seed=31)
    z = dense.sample_field(locs, xi, *th)
    ll0, ld0, q0 = dense.loglik_parts(locs, z, *th)
    S = scale(n, ld0, q0)
    res = {}
    for seed in (0, 12345, 12345):
        h = hcov.HCov(locs, th, eps=1e-8, leaf=64, eta=2.0, opts={"seed": seed})
        try:
            r = h.loglik(z)
        finally:
            h.close()
        assert abs(r[0] - ll0) / S < 1e-6
        if seed in res:
            assert r == res[seed]
        res[seed] = r
