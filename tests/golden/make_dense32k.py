"""Writes the dense FP64 oracle results for the n = 32,768 parity fixtures
(tests/golden/dense32k_*.npz).  Calls only the oracle (oracle.dense) and the
seeded input generators (workloads); run from the repository root:

    python tests/golden/make_dense32k.py

Each fixture holds the observation vector z (stored as float32; the oracle's
values below are computed from exactly the stored values), log|C|, the
quadratic form z^T C^{-1} z and the log-likelihood of Eq. (1), for:

* cfg2-32k: jittered 182 x 182 grid, 32,768 points kept (seed 7), Matérn
  sigma^2 1, ell 0.05, nu 1.5, nugget 1e-5 (the 128k jittered-grid
  configuration at a size the dense oracle holds);
* cfg4-32k: 32,768 uniform points (seed 32768), sigma^2 1, ell 0.08,
  nu 0.8, nugget 1e-4 (the 512k benchmark configuration's parameters).

z = L xi with the exact factor L (xi from the same generator).
"""
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy import linalg

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import dense  # noqa: E402

N = 32768
CASES = {
    "cfg2-32k": (lambda: workloads.jitter_grid(N, 182, seed=7), (1.0, 0.05, 1.5, 1e-5)),
    "cfg4-32k": (lambda: workloads.uniform(N, seed=N), (1.0, 0.08, 0.8, 1e-4)),
}


def assemble(locs, th):
    s2, ell, nu, nug = th
    C = np.empty((N, N))
    B = 1024

    def rows(i):
        C[i:i + B] = dense.cov_block(locs[i:i + B], locs, s2, ell, nu)

    with ThreadPoolExecutor(max_workers=os.cpu_count()) as ex:
        list(ex.map(rows, range(0, N, B)))
    C[np.diag_indices_from(C)] += nug
    return C


def main():
    for name, (gen, th) in CASES.items():
        t0 = time.time()
        locs, xi = gen()
        C = assemble(locs, th)
        L = dense.cholesky_torch(C)
        del C
        import torch
        z = (torch.from_numpy(L) @ torch.from_numpy(xi)).numpy().astype(np.float32)
        # Eq. (1) through the exact factor, as dense.loglik_parts composes it
        # (the matrix is assembled by blocks above: cov_block tiles cov_matrix)
        v = dense.forward_solve_torch(L, z.astype(np.float64))
        ld = dense.logdet_from_factor(L)
        q = float(v @ v)
        ll = -0.5 * N * math.log(2.0 * math.pi) - 0.5 * ld - 0.5 * q
        del L
        np.savez_compressed(os.path.join(HERE, f"dense32k_{name}.npz"), z=z, loglik=ll, logdet=ld, quad=q,
                            theta=np.array(th), n=N)
        print(f"{name}: loglik {ll:.10f} logdet {ld:.10f} quad {q:.10f} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
