"""Seeded synthetic inputs shared by the tests, the oracle checks and the
benchmark.  This module holds no arithmetic of the likelihood method: it only
draws locations, parameters, standard-normal vectors and arrival times with
NumPy's PCG64 generator (``numpy.random.default_rng``).

The paper's own data files are not available; these stand in for its
synthetic [0,1]^2 workloads (Sec. 5.1) with the shapes and sizes below.

Workloads (names are used by tests and ``bench.py``):

* ``uniform``   -- n i.i.d. points U([0,1]^2).
* ``jitter_grid`` -- centres ((i+1/2)h, (j+1/2)h) of a g x g grid, h = 1/g,
  each coordinate jittered by U(-0.4h, 0.4h); a seeded subset of n of the g^2
  points is kept in increasing grid order.
* ``mixture``   -- 70% U([0,1]^2) and 30% from 20 Gaussian clusters with
  sd 0.01 around centres drawn U([0,1]^2); cluster labels uniform.
* ``line``      -- n distinct points on the horizontal line y = 0.5 with
  sorted U(0,1) abscissae (the exact 1-D Markov checks).
* ``serving_stream`` -- requests with n log-uniform in [n_lo, n_hi],
  theta uniform in a box and Poisson arrival times.
"""
import math

import numpy as np


def uniform(n, seed=0):
    """Locations U([0,1]^2) and a standard-normal vector xi (same stream:
    locations first, then xi), as in the configuration with n=2000, seed 0."""
    rng = np.random.default_rng(seed)
    locs = rng.random((n, 2))
    xi = rng.standard_normal(n)
    return locs, xi


def jitter_grid(n, g, seed=0):
    """Jittered g x g grid, a seeded subset of n points (sorted grid order)."""
    if n > g * g:
        raise ValueError("n exceeds the grid")
    rng = np.random.default_rng(seed)
    h = 1.0 / g
    i, j = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    cx = (i.ravel() + 0.5) * h
    cy = (j.ravel() + 0.5) * h
    jit = rng.uniform(-0.4 * h, 0.4 * h, size=(g * g, 2))
    pts = np.stack([cx, cy], axis=1) + jit
    keep = np.sort(rng.choice(g * g, size=n, replace=False))
    xi = rng.standard_normal(n)
    return pts[keep], xi


def mixture(n, seed=0, n_clusters=20, frac=0.3, sd=0.01):
    """70/30 mixture of uniform points and Gaussian clusters (no clipping)."""
    rng = np.random.default_rng(seed)
    n_c = int(round(frac * n))
    n_u = n - n_c
    centres = rng.random((n_clusters, 2))
    lab = rng.integers(0, n_clusters, size=n_c)
    cl = centres[lab] + sd * rng.standard_normal((n_c, 2))
    un = rng.random((n_u, 2))
    locs = np.concatenate([un, cl], axis=0)
    xi = rng.standard_normal(n)
    return locs, xi


def line(n, seed=0, y0=0.5):
    """n points on y = y0 with sorted, distinct U(0,1) abscissae."""
    rng = np.random.default_rng(seed)
    x = np.sort(rng.random(n))
    if np.any(np.diff(x) <= 0):
        raise ValueError("duplicate abscissa drawn; change the seed")
    locs = np.stack([x, np.full(n, y0)], axis=1)
    xi = rng.standard_normal(n)
    return locs, xi


def theta_perturbations(theta, count, rel=0.10, seed=0):
    """``count`` parameter vectors (sigma2, ell, nu) each scaled by
    U(1-rel, 1+rel) around ``theta``."""
    rng = np.random.default_rng(seed)
    th = np.asarray(theta, dtype=np.float64)
    return th[None, :] * rng.uniform(1 - rel, 1 + rel, size=(count, len(th)))


def serving_stream(count=512, n_lo=1000, n_hi=64000, rate=1.0, seed=0,
                   sigma2=(0.5, 2.0), ell=(0.02, 0.3), nu=(0.3, 2.5)):
    """Request stream: list of dicts with arrival time (Poisson process of
    ``rate`` per second), n, theta and the seed of its own locations."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append(dict(id=r, arrival=float(t[r]), n=n,
                        sigma2=float(rng.uniform(*sigma2)),
                        ell=float(rng.uniform(*ell)),
                        nu=float(rng.uniform(*nu)),
                        seed=r))
    return out


def request_inputs(req):
    """Locations U([0,1]^2) and xi of one serving request (seed = request id)."""
    return uniform(req["n"], seed=1000 + req["seed"])
