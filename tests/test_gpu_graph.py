"""The factorisation sweep replayed from a captured HIP graph gives the same
bits as the sweep launched stage by stage: several replays with different
parameters, interleaved with other device work and synchronisations, each
compared with a context that launches every stage separately."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hcov():
    if not torch.cuda.is_available():
        pytest.skip("needs the GPU")
    from paper_1709_08625_amd import hcov as h
    return h


@pytest.mark.parametrize("n,leaf,eps", [(3000, 64, 1e-8), (9000, 128, 1e-7)])
def test_graph_replays_match_stage_launches(hcov, n, leaf, eps):
    locs, xi = workloads.uniform(n, seed=5)
    th0 = (1.0, 0.08, 0.8, 1e-4)
    G = hcov.HCov(locs, th0, eps=eps, leaf=leaf, opts={"use_graphs": 1})
    E = hcov.HCov(locs, th0, eps=eps, leaf=leaf, opts={"use_graphs": 0})
    z = np.random.default_rng(1).standard_normal(n)
    thetas = workloads.theta_perturbations(th0[:3], 4, rel=0.1, seed=3)
    junk = torch.zeros(1 << 20, device="cuda")
    for a, b, c in thetas:
        th = (float(a), float(b), float(c), th0[3])
        G.set_theta(th)
        E.set_theta(th)
        rg = G.loglik(z)
        junk.add_(1.0)                 # other device work between replays
        torch.cuda.synchronize()
        re = E.loglik(z)
        assert rg == re, (th, rg, re)
    # the plain factorisation (no fused right-hand side) is a second graph;
    # a new theta makes the contexts factorise again
    th = (1.1, 0.07, 0.9, th0[3])
    G.set_theta(th)
    E.set_theta(th)
    G.cholesky()
    E.cholesky()
    assert G.logdet() == E.logdet()
    # every factorisation of G (the retries of saturated sketches included) replays
    st = G.stats()
    assert st["n_graph_replays"] == 5 + st["n_sketch_retries"]
    assert st["n_sketch_retries"] == E.stats()["n_sketch_retries"]
    assert E.stats()["n_graph_replays"] == 0
    G.close()
    E.close()
