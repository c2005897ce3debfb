"""Reference Nelder-Mead simplex minimiser (oracle; test infrastructure only).

The paper maximises the likelihood with a derivative-free simplex search over
theta (Sec. 5 and the driver listing of Appendix B: initial steps
(0.02, 0.04, 0.01) for (nu, ell, sigma^2), at most 200 iterations, simplex-size
test 1e-5).  This is the classic method of Nelder & Mead (1965) with
reflection 1, expansion 2, contraction 1/2 and shrink 1/2; the initial simplex
is x0 and x0 + step_k e_k.  Ties are broken by vertex index (stable sort).

It minimises f, so a likelihood driver passes f = -L.
"""
import numpy as np


def nelder_mead(f, x0, steps, max_evals=200, size_tol=1e-5):
    """Return (x_best, f_best, n_evals, history) with history the list of
    (x, f) of every evaluation in order."""
    x0 = np.asarray(x0, dtype=np.float64)
    d = len(x0)
    hist = []

    def F(x):
        v = float(f(x))
        hist.append((x.copy(), v))
        return v

    simplex = [x0.copy()] + [x0 + steps[k] * np.eye(d)[k] for k in range(d)]
    fv = [F(x) for x in simplex]
    while len(hist) < max_evals:
        order = np.argsort(fv, kind="stable")
        simplex = [simplex[i] for i in order]
        fv = [fv[i] for i in order]
        centroid = np.mean(simplex[:-1], axis=0)
        size = max(np.linalg.norm(x - centroid) for x in simplex)
        if size < size_tol:
            break
        worst = simplex[-1]
        xr = centroid + (centroid - worst)
        fr = F(xr)
        if fr < fv[0]:
            if len(hist) >= max_evals:
                simplex[-1], fv[-1] = xr, fr
                break
            xe = centroid + 2.0 * (centroid - worst)
            fe = F(xe)
            if fe < fr:
                simplex[-1], fv[-1] = xe, fe
            else:
                simplex[-1], fv[-1] = xr, fr
        elif fr < fv[-2]:
            simplex[-1], fv[-1] = xr, fr
        else:
            if len(hist) >= max_evals:
                break
            if fr < fv[-1]:
                xc = centroid + 0.5 * (xr - centroid)
            else:
                xc = centroid + 0.5 * (worst - centroid)
            fc = F(xc)
            if fc < min(fr, fv[-1]):
                simplex[-1], fv[-1] = xc, fc
            else:
                for i in range(1, d + 1):
                    if len(hist) >= max_evals:
                        break
                    simplex[i] = simplex[0] + 0.5 * (simplex[i] - simplex[0])
                    fv[i] = F(simplex[i])
    b = int(np.argmin(fv))
    return simplex[b], fv[b], len(hist), hist
