"""The library's Nelder-Mead (host code of the outer loop) against the
oracle's independent implementation of the same published method: identical
evaluation histories on deterministic objectives (CPU only)."""
import numpy as np
import pytest

from oracle.nelder_mead import nelder_mead
from paper_1709_08625_amd import hcov


@pytest.mark.parametrize("fname", ["quad", "rosen", "flat"])
def test_library_nm_matches_oracle_history(fname):
    funcs = {
        "quad": (lambda x: float(np.sum((x - np.array([0.3, -1.2, 2.0])) ** 2 * np.array([1.0, 3.0, 0.5]))),
                 np.zeros(3), [0.5, 0.5, 0.5], 300),
        "rosen": (lambda x: float(100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2), np.array([-1.2, 1.0]),
                  [0.1, 0.1], 400),
        "flat": (lambda x: float(abs(x[0] - 0.5) + 1e-3 * x[1] ** 2 + (x[2] - 1) ** 4), np.array([0.8, 0.08, 1.1]),
                 [0.02, 0.04, 0.01], 30),
    }
    f, x0, steps, cap = funcs[fname]
    xo, fo, no, ho = nelder_mead(f, x0, steps, max_evals=cap, size_tol=1e-7)
    xl, fl, nl, hl = hcov.nm_minimize(f, x0, steps, max_evals=cap, size_tol=1e-7)
    assert no == nl
    for (a, fa), (b, fb) in zip(ho, hl):
        assert np.array_equal(a, b) and fa == fb
    assert np.array_equal(xo, xl) and fo == fl


def test_library_nm_rejects_bad_arguments():
    with pytest.raises(hcov.HcovError):
        hcov.nm_minimize(lambda x: 0.0, np.zeros(3), [0.1, 0.1, 0.1], max_evals=0)


@pytest.mark.parametrize("move", ["reflection", "expansion", "outside", "inside", "shrink"])
def test_library_nm_single_moves_by_hand(move):
    # the hand-worked single moves of the method (tests/test_oracle_nm.py),
    # checked on the library directly so that a mistake shared with the
    # oracle's implementation cannot hide
    from tests.test_oracle_nm import MOVES

    f, cap, want = MOVES[move]
    _, _, n, hist = hcov.nm_minimize(f, np.zeros(2), [1.0, 1.0], max_evals=cap, size_tol=0.0)
    assert [tuple(float(c) for c in x) for x, _ in hist] == want
