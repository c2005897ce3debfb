"""Pins of the reference Nelder-Mead minimiser (CPU only)."""
import numpy as np
import pytest

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


# ---------------------------------------------------------------- single moves, by hand
# Nelder & Mead (1965) on the 2-D simplex v0 = (0,0), v1 = (1,0), v2 = (0,1)
# (x0 = 0, steps (1, 1)).  Each case fixes f so that one move happens; the
# expected evaluation sequence is worked out by hand from the method's
# definition (reflection xr = c + (c - w), expansion xe = c + 2 (c - w),
# outside contraction c + (xr - c)/2, inside contraction c + (w - c)/2, shrink
# v_i <- v_best + (v_i - v_best)/2, c the centroid of all but the worst w),
# every coordinate a dyadic fraction so the points are exact.
V0, V1, V2 = (0.0, 0.0), (1.0, 0.0), (0.0, 1.0)


def _table(values, default):
    return lambda x: values.get((float(x[0]), float(x[1])), default)


def _run(f, max_evals):
    _, _, n, hist = nelder_mead(f, np.zeros(2), [1.0, 1.0], max_evals=max_evals, size_tol=0.0)
    return [tuple(float(c) for c in x) for x, _ in hist]


MOVES = {
    # f = (x - 1)^2 + (y + 0.3)^2: order v1 (0.09) < v0 (1.09) < v2 (2.69);
    # c = (0.5, 0), xr = (1, -1) with f = 0.49 in [f(v1), f(v0)): reflection kept
    "reflection": (lambda x: (x[0] - 1.0) ** 2 + (x[1] + 0.3) ** 2, 4, [V0, V1, V2, (1.0, -1.0)]),
    # f = x + 2y: order v0 (0) < v1 (1) < v2 (2); xr = (1, -1), f = -1 < 0:
    # expansion xe = (1.5, -2), f = -2.5 < -1 is kept
    "expansion": (lambda x: x[0] + 2.0 * x[1], 5, [V0, V1, V2, (1.0, -1.0), (1.5, -2.0)]),
    # f = (x - 0.6)^2 + (y + 0.3)^2: order v1 (0.25) < v0 (0.45) < v2 (2.05);
    # xr = (1, -1), f = 0.65 in [f(v0), f(v2)): outside contraction
    # (0.75, -0.5), f = 0.0625 kept
    "outside": (lambda x: (x[0] - 0.6) ** 2 + (x[1] + 0.3) ** 2, 5, [V0, V1, V2, (1.0, -1.0), (0.75, -0.5)]),
    # f = (x - 0.3)^2 + (y - 0.9)^2: order v2 (0.10) < v0 (0.90) < v1 (1.30);
    # c = (0, 0.5), w = v1, xr = (-1, 1), f = 1.70 >= f(w): inside contraction
    # (0.5, 0.25), f = 0.4625 kept
    "inside": (lambda x: (x[0] - 0.3) ** 2 + (x[1] - 0.9) ** 2, 5, [V0, V1, V2, (-1.0, 1.0), (0.5, 0.25)]),
    # tabulated f: v0 1 < v1 2 < v2 3; xr = (1, -1) -> 10 (>= f(w)); inside
    # contraction (0.25, 0.5) -> 5 >= min(10, 3): shrink towards v0, v1 -> (0.5, 0),
    # v2 -> (0, 0.5)
    "shrink": (_table({V0: 1.0, V1: 2.0, V2: 3.0, (1.0, -1.0): 10.0, (0.25, 0.5): 5.0}, 7.0), 7,
               [V0, V1, V2, (1.0, -1.0), (0.25, 0.5), (0.5, 0.0), (0.0, 0.5)]),
}


@pytest.mark.parametrize("move", sorted(MOVES))
def test_single_move_by_hand(move):
    f, cap, want = MOVES[move]
    assert _run(f, cap) == want


def test_shrink_then_new_order():
    # after the shrink of the tabulated case the simplex is v0 = (0,0) (f 1),
    # (0.5, 0) and (0, 0.5) (both 7, the default): order v0, (0.5,0), (0,0.5);
    # c = (0.25, 0), w = (0, 0.5), the next reflection is (0.5, -0.5)
    f, _, want = MOVES["shrink"]
    assert _run(f, 8) == want + [(0.5, -0.5)]
