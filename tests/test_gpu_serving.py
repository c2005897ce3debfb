"""Serving (request loop with concurrent slots, memory admission, resident
data sets): every result is bit-identical to the same evaluation run alone.
Inputs follow the serving workload: n log-uniform, uniform locations,
theta uniform in the stated boxes; z is a standard normal vector."""
import numpy as np
import pytest

import workloads
from paper_1709_08625_amd import hcov

pytestmark = pytest.mark.gpu


def _requests(count, seed, n_lo=800, n_hi=6000, model_z=False):
    # z = xi (the serving workload) or, for comparisons with the dense oracle,
    # a sample z = L xi of the request's own model (with white noise, q is
    # dominated by the nugget-sized eigenvalues of these smooth kernels and is
    # conditioned far worse than the likelihoods the method is asked for)
    out = []
    rng = np.random.default_rng(seed)
    for i in range(count):
        n = int(np.floor(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        locs, z = workloads.uniform(n, seed=1000 + i)
        th = (rng.uniform(0.5, 2.0), rng.uniform(0.02, 0.3), rng.uniform(0.3, 2.5), 1e-4)
        if model_z:
            from oracle import dense
            z = dense.sample_field(locs, z, *th)
        out.append((locs, z, th))
    return out


def _alone(locs, z, th, eps, leaf, eta):
    H = hcov.HCov(locs, th, eps=eps, leaf=leaf, eta=eta)
    try:
        return H.loglik(z)
    finally:
        H.close()


def test_mix_equals_alone():
    # eps 1e-9, the block accuracy at which the FP64 tolerance 1e-6 of S is
    # stated (these smooth kernels, nu up to 2.5 with ell up to 0.3 and nugget
    # 1e-4, have condition numbers ~1e7; at eps 1e-8 one request lands at
    # 1.03e-6)
    eps, leaf, eta = 1e-9, 64, 2.0
    reqs = _requests(10, seed=3, model_z=True)
    alone = [_alone(l, z, th, eps, leaf, eta) for l, z, th in reqs]
    S = hcov.Server(slots=4)
    try:
        tickets = [S.submit(z, th, locs=l, eps=eps, leaf=leaf, eta=eta) for l, z, th in reqs]
        res = [S.wait(t) for t in tickets]
    finally:
        S.close()
    for (ll, ld, q), r in zip(alone, res):
        assert r["status"] == 0
        assert (r["loglik"], r["logdet"], r["quad"]) == (ll, ld, q)
        assert r["latency_ms"] >= r["service_ms"] > 0.0
    # and every served result is the dense FP64 likelihood of its request to
    # the FP64 tolerance (requests of n <= 6000 here; theta spans the serving
    # boxes: nu in [0.3, 2.5], ell in [0.02, 0.3])
    import math
    from oracle import dense
    for (l, z, th), r in zip(reqs, res):
        ll0, ld0, q0 = dense.loglik_parts(l, z, *th)
        S = 0.5 * len(z) * math.log(2 * math.pi) + abs(ld0) / 2 + q0 / 2
        assert abs(r["loglik"] - ll0) / S < 1e-6, (len(z), th, r["loglik"], ll0)


def test_small_budget_still_serves_one_at_a_time():
    eps, leaf, eta = 1e-8, 64, 2.0
    reqs = _requests(3, seed=5, n_hi=3000)
    alone = [_alone(l, z, th, eps, leaf, eta) for l, z, th in reqs]
    S = hcov.Server(slots=3, mem_budget=1)
    try:
        tickets = [S.submit(z, th, locs=l, eps=eps, leaf=leaf, eta=eta) for l, z, th in reqs]
        res = [S.wait(t) for t in tickets]
        with pytest.raises(hcov.HcovError):
            S.poll(tickets[0])       # a result is handed out once
    finally:
        S.close()
    for (ll, ld, q), r in zip(alone, res):
        assert (r["loglik"], r["logdet"], r["quad"]) == (ll, ld, q)


def test_resident_dataset_matches_context():
    eps, leaf, eta = 1e-8, 64, 2.0
    locs, z = workloads.uniform(4000, seed=11)
    thetas = [(1.0, 0.1, 0.8, 1e-4), (1.3, 0.07, 1.1, 1e-4), (0.8, 0.15, 0.6, 1e-4)]
    H = hcov.HCov(locs, thetas[0], eps=eps, leaf=leaf, eta=eta)
    try:
        ref = []
        for th in thetas:
            H.set_theta(th)
            ref.append(H.loglik(z))
    finally:
        H.close()
    S = hcov.Server(slots=2)
    try:
        ds = S.dataset(locs, thetas[0], eps=eps, leaf=leaf, eta=eta)
        tickets = [S.submit(z, th, dataset=ds) for th in thetas]
        other = _requests(2, seed=9, n_hi=2000)
        t2 = [S.submit(zz, th, locs=l, eps=eps, leaf=leaf, eta=eta) for l, zz, th in other]
        res = [S.wait(t) for t in tickets]
        res2 = [S.wait(t) for t in t2]
        S.release(ds)
        with pytest.raises(hcov.HcovError):
            S.submit(z, thetas[0], dataset=ds)
    finally:
        S.close()
    for (ll, ld, q), r in zip(ref, res):
        assert (r["loglik"], r["logdet"], r["quad"]) == (ll, ld, q)
    for (l, zz, th), r in zip(other, res2):
        assert (r["loglik"], r["logdet"], r["quad"]) == _alone(l, zz, th, eps, leaf, eta)


# ------------------------------------------------------------------ failures
def test_poisoned_request_fails_alone():
    # one request in the mix has two coincident locations and no nugget (an
    # exactly singular C: Sec. 3 names duplicate locations as the cause of a
    # failing factorisation); it reports HCOV_ENOTSPD while every other
    # request of the mix returns what it returns alone, bit for bit
    eps, leaf, eta = 1e-8, 64, 2.0
    reqs = _requests(5, seed=13, n_hi=3000)
    locs, z = workloads.uniform(1500, seed=77)
    locs[40] = locs[7]
    bad = (locs, z, (1.0, 0.1, 0.5, 0.0))
    mix = reqs[:2] + [bad] + reqs[2:]
    alone = [_alone(l, zz, th, eps, leaf, eta) for l, zz, th in reqs]
    S = hcov.Server(slots=3)
    try:
        tickets = [S.submit(zz, th, locs=l, eps=eps, leaf=leaf, eta=eta) for l, zz, th in mix]
        res = [S.wait(t) for t in tickets]
    finally:
        S.close()
    assert res[2]["status"] == hcov.ENOTSPD
    good = res[:2] + res[3:]
    for (ll, ld, q), r in zip(alone, good):
        assert r["status"] == 0
        assert (r["loglik"], r["logdet"], r["quad"]) == (ll, ld, q)


def test_memory_cap_rejects_only_what_exceeds_it():
    # opts.mem_cap_bytes: a build whose planned device memory exceeds the cap
    # fails with HCOV_ENOMEM before it allocates; below the cap it runs.  The
    # cap is set between the footprints of a small and a large request, and
    # the server applies it per request
    eps, leaf, eta = 1e-8, 64, 2.0
    small = _requests(1, seed=21, n_lo=900, n_hi=901)[0]
    large = _requests(1, seed=22, n_lo=12000, n_hi=12001)[0]
    foot = []
    for l, zz, th in (small, large):
        H = hcov.HCov(l, th, eps=eps, leaf=leaf, eta=eta)
        try:
            foot.append(H.stats()["bytes_device"])
        finally:
            H.close()
    assert foot[1] > 4 * foot[0]
    cap = 2 * foot[0]
    with pytest.raises(hcov.HcovError) as e:
        hcov.HCov(large[0], large[2], eps=eps, leaf=leaf, eta=eta, opts={"mem_cap_bytes": cap})
    assert e.value.code == hcov.ENOMEM
    S = hcov.Server(slots=2, opts={"mem_cap_bytes": cap})
    try:
        t = [S.submit(zz, th, locs=l, eps=eps, leaf=leaf, eta=eta) for l, zz, th in (small, large)]
        r = [S.wait(x) for x in t]
    finally:
        S.close()
    assert r[0]["status"] == 0
    assert (r[0]["loglik"], r[0]["logdet"], r[0]["quad"]) == _alone(*small, eps, leaf, eta)
    assert r[1]["status"] == hcov.ENOMEM
