"""Parameter identification at small scale (GPU): Z0 = L~ xi drawn from the
H-Cholesky factor (Sec. 5.1), replicate subsets fitted by the library's
Nelder-Mead search (the experiment of Fig. 9, reduced: n0 = 30,000, two
subset sizes, two replicates, 30 evaluations per fit)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_parameter_identification_small():
    from paper_1709_08625_amd import paramid
    locs0, xi0 = workloads.uniform(30000, seed=3)
    z0 = paramid.draw_field(locs0, xi0)
    # the field has the model's marginal variance sigma^2 + nugget, up to the
    # sampling error of a correlated field (effective sample size ~ 1/ell^2)
    v = float(np.var(z0))
    assert 0.5 < v < 1.6, v
    start = (1.2, 0.0864 * 0.8, 0.55)
    fits = paramid.identify(locs0, z0, [1000, 3000], 2, start, max_evals=30)
    assert len(fits) == 4
    for f in fits:
        s2, ell, nu = f["theta"]
        print(f"n={f['n']} r={f['replicate']}: sigma2 {s2:.3f} ell {ell:.4f} nu {nu:.3f} "
              f"(-L {-f['loglik']:.2f} from {f['start_negll']:.2f})")
        assert np.isfinite(f["loglik"]) and f["evals"] == 30
        assert -f["loglik"] <= f["start_negll"]          # the search did not get worse than its start
        assert 0.1 < s2 < 10 and 0.005 < ell < 1.0 and 0.05 < nu < 5
    summ = paramid.summarise(fits)
    assert set(summ) == {"1000", "3000"}
