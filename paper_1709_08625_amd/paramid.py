"""Parameter identification on synthetic data (Sec. 5.1 and the appendix on
the maximum of the log-likelihood, Fig. 9).

A field Z0 = L~ xi is drawn once at n0 locations from the H-Cholesky factor
of C(theta*) (theta* = (ell, nu, sigma^2) = (0.0864, 0.5, 1.0) in the paper);
M replicate data sets of n points are sampled from (locations, Z0) for each
n, and every replicate is fitted by the library's Nelder-Mead search over
(sigma^2, ell, nu) on the H-likelihood (hcov_fit).  The spread of the
estimates over the replicates should shrink as n grows.

Orchestration only: every likelihood evaluation, the factorisation that
draws Z0 and the simplex search run in the HIP library.
"""
import time

import numpy as np

from . import hcov

TRUTH = (1.0, 0.0864, 0.5)     # (sigma^2, ell, nu)


def draw_field(locs0, xi0, truth=TRUTH, nugget=1e-4, eps=1e-7, leaf=128, eta=2.0, stream=None):
    """Z0 = P^T L~ xi0 at the given locations (external order)."""
    H = hcov.HCov(locs0, (*truth, nugget), eps=eps, leaf=leaf, eta=eta, stream=stream)
    try:
        H.cholesky()
        return H.sample(xi0[H.perm()])
    finally:
        H.close()


def identify(locs0, z0, sizes, replicates, start, nugget=1e-4, eps=1e-7, leaf=64, eta=2.0, max_evals=60,
             size_tol=1e-6, seed=1, progress=None):
    """Replicate fits: for each n in `sizes`, `replicates` random subsets of
    n of the n0 points (without replacement, seeded), each fitted from
    `start` = (sigma^2, ell, nu).  Returns a list of dicts per fit."""
    rng = np.random.default_rng(seed)
    n0 = len(z0)
    out = []
    for n in sizes:
        for r in range(replicates):
            idx = np.sort(rng.choice(n0, n, replace=False))
            t0 = time.perf_counter()
            H = hcov.HCov(locs0[idx], (*start, nugget), eps=eps, leaf=leaf, eta=eta)
            try:
                th, ll, ne, hist = H.fit(z0[idx], np.asarray(start, dtype=np.float64), nugget,
                                         max_evals=max_evals, size_tol=size_tol)
            finally:
                H.close()
            dt = time.perf_counter() - t0
            out.append({"n": int(n), "replicate": r, "theta": [float(x) for x in th], "loglik": float(ll),
                        "evals": int(ne), "seconds": dt, "start_negll": float(hist[0][1])})
            if progress:
                progress(f"n={n} replicate {r}: sigma2 {th[0]:.4f} ell {th[1]:.4f} nu {th[2]:.4f} "
                         f"({ne} evaluations, {dt:.1f} s)")
    return out


def summarise(fits):
    """Mean and standard deviation of each estimate per n."""
    res = {}
    for n in sorted({f["n"] for f in fits}):
        th = np.array([f["theta"] for f in fits if f["n"] == n])
        res[str(n)] = {"replicates": len(th),
                       "mean": {"sigma2": float(th[:, 0].mean()), "ell": float(th[:, 1].mean()),
                                "nu": float(th[:, 2].mean())},
                       "sd": {"sigma2": float(th[:, 0].std()), "ell": float(th[:, 1].std()),
                              "nu": float(th[:, 2].std())}}
    return res
