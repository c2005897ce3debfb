"""Pins of the reference Nelder-Mead minimiser (CPU only)."""
import numpy as np

from oracle.nelder_mead import nelder_mead


def test_quadratic_minimum():
    c = np.array([0.3, -1.2, 2.0])
    f = lambda x: float(np.sum((x - c) ** 2 * np.array([1.0, 3.0, 0.5])))
    x, fx, n, hist = nelder_mead(f, np.zeros(3), [0.5, 0.5, 0.5], max_evals=600, size_tol=1e-9)
    assert np.max(np.abs(x - c)) < 1e-6 and fx < 1e-11
    assert n == len(hist) <= 600


def test_rosenbrock_2d():
    f = lambda x: float(100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2)
    x, fx, n, _ = nelder_mead(f, np.array([-1.2, 1.0]), [0.1, 0.1], max_evals=2000, size_tol=1e-10)
    assert np.max(np.abs(x - 1.0)) < 1e-4


def test_eval_cap_is_respected():
    f = lambda x: float(np.sum(x ** 2))
    _, _, n, hist = nelder_mead(f, np.ones(3), [0.02, 0.04, 0.01], max_evals=30)
    assert n == len(hist) <= 30
