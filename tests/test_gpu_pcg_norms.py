"""Kept C~, PCG quadratic form, factor products and accuracy norms (GPU).

* The quadratic form z^T C~^{-1} z by conjugate gradients on C~ with the
  H-Cholesky factor as preconditioner (the listing of Appendix B: CG with the
  factor, tolerance 1e-6) against the dense FP64 oracle.
* The kept copy of C~ gives the same H-matvec after the factorisation as
  before it; L~ L~^T x and the H-solves are inverse to each other.
* Power-iteration norms (Sec. 3, the error columns of Tables 2, 3 and 5)
  against the same norms computed densely from the matrices the library
  represents (C~ and L~ L~^T extracted column by column).
* Fixed-rank H-matrices (Tables 2 and 3): KLD, ||C - C~||_2 and
  ||C (L~L~^T)^{-1} - I||_2 fall as the rank k grows (the shape of Table 2;
  the paper does not state n or the block structure, so its values are not
  matched: parity unpinned for the table's numbers).
"""
import math

import numpy as np
import pytest

import workloads
from oracle import dense

pytestmark = pytest.mark.gpu


def _hc():
    from paper_1709_08625_amd import hcov
    return hcov


def scale(n, ld, q):
    return 0.5 * n * math.log(2 * math.pi) + abs(ld) / 2 + q / 2


@pytest.mark.parametrize("eps", [1e-7, 1e-5])
def test_pcg_quadratic_form_against_dense(eps):
    hcov = _hc()
    n, th = 3000, (1.0, 0.08, 0.8, 1e-4)
    locs, xi = workloads.uniform(n, seed=31)
    z = dense.sample_field(locs, xi, *th)
    ll0, ld0, q0 = dense.loglik_parts(locs, z, *th)
    S = scale(n, ld0, q0)
    hd = hcov.HCov(locs, th, eps=eps, leaf=64, eta=2.0)
    lld, ldd, qd = hd.loglik(z)
    hd.close()
    hp = hcov.HCov(locs, th, eps=eps, leaf=64, eta=2.0, opts={"quad_mode": hcov.QUAD_PCG})
    llp, ldp, qp = hp.loglik(z)
    st = hp.stats()
    hp.close()
    print(f"eps={eps}: direct q err {abs(qd - q0) / S:.2e}, PCG q err {abs(qp - q0) / S:.2e} "
          f"({st['pcg_iters']} iterations, residual {st['pcg_relres']:.1e}); logdet err {abs(ldp - ld0) / S:.2e}")
    # the preconditioner's own solution may already meet the tolerance (0 iterations)
    assert st["pcg_relres"] <= 1e-6 and 0 <= st["pcg_iters"] <= 150
    assert ldp == ldd                       # the log-determinant still comes from the factor
    # CG on C~ replaces the factor's error in q by the assembly's (C~ vs C):
    # both are of the block accuracy, neither is always the smaller
    assert abs(llp - ll0) / S < (1e-6 if eps <= 1e-7 else 1e-4)
    assert abs(qp - q0) / S < (1e-6 if eps <= 1e-7 else 1e-4)


def test_kept_matrix_products():
    hcov = _hc()
    n, th = 900, (1.2, 0.1, 1.3, 1e-3)
    locs, _ = workloads.uniform(n, seed=32)
    h = hcov.HCov(locs, th, eps=1e-9, leaf=32, eta=2.0, opts={"keep_matrix": 1})
    x = np.random.default_rng(1).standard_normal(n)
    y0 = h.matvec(x)
    h.cholesky()
    assert np.array_equal(h.matvec(x), y0)           # the kept copy is the assembled C~
    m = h.factor_matvec(x)
    C = dense.cov_matrix(locs, *th)
    assert np.linalg.norm(m - C @ x) / np.linalg.norm(C @ x) < 1e-7
    back = h.solve(m)                                 # (L~L~^T)^{-1} L~L~^T x = x
    assert np.linalg.norm(back - x) / np.linalg.norm(x) < 1e-9
    # exact on-the-fly products against the oracle's dense matrix
    e = h.exact_matvec(x)
    assert np.linalg.norm(e - C @ x) / np.linalg.norm(C @ x) < 1e-13
    h.close()


def _dense_of(op, n):
    return np.column_stack([op(np.eye(n)[:, j]) for j in range(n)])


def test_error_norms_against_dense():
    hcov = _hc()
    n, th = 500, (1.0, 0.15, 0.5, 1e-3)
    locs, _ = workloads.uniform(n, seed=33)
    h = hcov.HCov(locs, th, eps=1e-4, leaf=32, eta=2.0, opts={"keep_matrix": 1})
    h.cholesky()
    Ct = _dense_of(h.matvec, n)
    M = _dense_of(h.factor_matvec, n)
    C = dense.cov_matrix(locs, *th)
    ref_c = np.linalg.norm(Ct, 2)
    ref_f = np.linalg.norm(Ct - M, 2)
    ref_i = np.linalg.norm(np.eye(n) - np.linalg.solve(M, Ct), 2)
    ref_e = np.linalg.norm(C - Ct, 2)
    ref_ei = np.linalg.norm(C @ np.linalg.inv(M) - np.eye(n), 2)
    nc, nf, ni = h.error_norms(iters=60, seed=3)
    ec, eci = h.exact_norms(iters=60, seed=5)
    h.close()
    print(f"||C~|| {nc:.4e}/{ref_c:.4e}  ||C~-LL'|| {nf:.3e}/{ref_f:.3e}  ||I-(LL')^-1 C~|| {ni:.3e}/{ref_i:.3e}  "
          f"||C-C~|| {ec:.3e}/{ref_e:.3e}  ||C(LL')^-1-I|| {eci:.3e}/{ref_ei:.3e}")
    for est, ref in [(nc, ref_c), (nf, ref_f), (ni, ref_i), (ec, ref_e), (eci, ref_ei)]:
        # power iteration gives lower bounds converging to the norm
        assert 0.8 * ref <= est <= ref * (1 + 1e-6) + 1e-300


def test_fixed_rank_errors_fall_with_rank():
    # the shape of Table 2: Matérn nu = 1/2, ell = 0.25, sigma^2 = 1 on [0,1]^2,
    # nugget 0, fixed-rank blocks of rank k
    hcov = _hc()
    n, th = 1024, (1.0, 0.25, 0.5, 0.0)
    locs, _ = workloads.uniform(n, seed=34)
    C = dense.cov_matrix(locs, *th)
    _, ldC = np.linalg.slogdet(C)
    rows = []
    for k in (3, 5, 8, 12):
        h = hcov.HCov(locs, th, eps=1e-15, leaf=32, eta=2.0, opts={"keep_matrix": 1, "fixed_rank": k})
        h.cholesky()
        Ct = _dense_of(h.matvec, n)
        Ct = 0.5 * (Ct + Ct.T)
        _, ldt = np.linalg.slogdet(Ct)
        kld = 0.5 * (np.trace(np.linalg.solve(Ct, C)) - n - (ldC - ldt))
        ec, eci = h.exact_norms(iters=40, seed=7)
        assert h.stats()["max_rank_seen"] <= k
        h.close()
        rows.append((k, kld, ec, eci))
        print(f"k={k}: KLD {kld:.2e}  ||C-C~|| {ec:.2e}  ||C (LL')^-1 - I|| {eci:.2e}")
    for (k0, a0, b0, c0), (k1, a1, b1, c1) in zip(rows, rows[1:]):
        assert a1 < a0 and b1 < b0 and c1 < c0, (k0, k1)
