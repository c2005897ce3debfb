"""Pins of the CPU oracle against what the paper and mathematics fix
(closed forms, brute force, invariants, independent high-precision values).
CPU only."""
import math

import numpy as np
import pytest

import workloads
from oracle import brute, dense, markov, matern


# ---------------------------------------------------------------- Matérn, Eq. (3)

@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_matern_half_integer_closed_forms(nu):
    # Sec. 2.1: nu = 1/2 is the exponential kernel; the half-integer cases are
    # elementary.  Catches a wrong 2^(nu-1) Gamma(nu) normalisation or a
    # sqrt(2 nu) rescaling of the argument.
    h = np.linspace(1e-6, 3.0, 4001)
    for ell in (0.05, 0.1, 0.3):
        a = matern.matern(h, 1.7, ell, nu)
        b = matern.matern_half_integer(h, 1.7, ell, nu)
        np.testing.assert_allclose(a, b, rtol=2e-14, atol=1e-300)


def test_matern_zero_distance_is_variance():
    for nu in (0.3, 0.8, 1.5, 2.2):
        assert matern.matern(np.array([0.0]), 2.5, 0.1, nu)[0] == 2.5
        # the h -> 0 limit of Eq. (3) approaches sigma^2 continuously
        # (the deviation from sigma^2 scales like x^(2 min(nu, 1)))
        x = 1e-9 / 0.1
        v = matern.matern(np.array([1e-9]), 2.5, 0.1, nu)[0]
        assert abs(2.5 - v) < (10 * x ** (2 * min(nu, 1.0)) + 1e-15) * 2.5


def test_scipy_kv_against_mpmath():
    # the library step of the oracle (scipy.special.kv) against an independent
    # 50-digit evaluation on nu in [0.3, 2.5], x in [1e-8, 700]; scipy's own
    # accuracy near its branch switch (x ~ 2) is a few 1e-14 relative, and it
    # flushes values below ~1e-305 to zero
    from scipy import special

    nus = [0.3, 0.5, 0.8, 1.0, 1.37, 1.5, 2.0, 2.2, 2.5]
    xs = [1e-8, 1e-4, 0.01, 0.3, 1.0, 1.99, 2.01, 5.0, 17.0, 60.0, 300.0, 700.0]
    for nu in nus:
        for x in xs:
            ref = float(matern.besselk_mp(nu, x))
            got = float(special.kv(nu, x))
            assert abs(got - ref) <= 1e-13 * abs(ref) + 1e-300, (nu, x, got, ref)


def test_matern_against_mpmath():
    rng = np.random.default_rng(3)
    for _ in range(40):
        nu = rng.uniform(0.3, 2.5)
        ell = rng.uniform(0.02, 0.3)
        h = rng.uniform(0, 1.5)
        got = matern.matern(np.array([h]), 1.3, ell, nu)[0]
        ref = float(matern.matern_mp(h, 1.3, ell, nu))
        assert abs(got - ref) <= 1e-13 * max(abs(ref), 1e-300), (nu, ell, h)


# ---------------------------------------------------------------- Eq. (1) dense

def test_loglik_n1_closed_form():
    s2, tau2, z = 1.7, 1e-3, 0.37
    ll = dense.loglik(np.array([[0.2, 0.4]]), np.array([z]), s2, 0.1, 0.8, tau2)
    v = s2 + tau2
    ref = -0.5 * math.log(2 * math.pi) - 0.5 * math.log(v) - z * z / (2 * v)
    assert abs(ll - ref) < 1e-15


def test_loglik_n2_closed_form():
    locs = np.array([[0.1, 0.2], [0.4, 0.6]])
    z = np.array([0.3, -1.1])
    s2, ell, nu, tau2 = 1.2, 0.3, 0.5, 1e-4
    c = s2 * math.exp(-0.5 / ell)          # |s1 - s2| = 0.5, nu = 1/2
    a = s2 + tau2
    det = a * a - c * c
    quad = (a * z[0] ** 2 - 2 * c * z[0] * z[1] + a * z[1] ** 2) / det
    ref = -math.log(2 * math.pi) - 0.5 * math.log(det) - 0.5 * quad
    assert abs(dense.loglik(locs, z, s2, ell, nu, tau2) - ref) < 1e-14


@pytest.mark.parametrize("n,nu", [(3, 0.5), (5, 0.8), (8, 1.5), (8, 2.2)])
def test_loglik_brute_force_mp(n, nu):
    locs, xi = workloads.uniform(n, seed=n)
    z = xi
    ll, ld, q = dense.loglik_parts(locs, z, 1.1, 0.2, nu, 1e-4)
    llm, ldm, qm = brute.loglik_mp(locs, z, 1.1, 0.2, nu, 1e-4)
    assert abs(ld - float(ldm)) < 1e-10 * max(1.0, abs(float(ldm)))
    assert abs(q - float(qm)) < 1e-10 * max(1.0, abs(float(qm)))
    assert abs(ll - float(llm)) < 1e-10 * max(1.0, abs(float(llm)))


def test_paper_input_example_brute_force():
    # the three-point input file printed in Sec. 4 (tests/golden)
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "paper_input_example.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    n = int(rows[0][0])
    data = np.array([[float(v) for v in r] for r in rows[1:1 + n]])
    assert data.shape == (3, 3)
    locs, z = data[:, :2], data[:, 2]
    ll = dense.loglik(locs, z, 1.0, 0.1, 0.5, 1e-4, own=True)
    llm = brute.loglik_mp(locs, z, 1.0, 0.1, 0.5, 1e-4)[0]
    assert abs(ll - float(llm)) < 1e-9 * abs(float(llm))


def test_own_cholesky_matches_lapack():
    locs, _ = workloads.uniform(400, seed=1)
    C = dense.cov_matrix(locs, 1.0, 0.1, 0.8, 1e-4)
    L1 = dense.cholesky_unblocked(C)
    L2 = dense.cholesky_lapack(C)
    assert np.max(np.abs(L1 - L2)) < 1e-9
    np.testing.assert_allclose(L1 @ L1.T, C, atol=1e-12)
    z = np.random.default_rng(0).standard_normal(400)
    v1 = dense.forward_solve_unblocked(L1, z)
    v2 = dense.forward_solve_lapack(L2, z)
    assert np.max(np.abs(v1 - v2)) < 1e-6 * np.max(np.abs(v2))


def test_cov_symmetric_spd_and_nugget_on_diagonal():
    locs, _ = workloads.uniform(300, seed=2)
    C0 = dense.cov_matrix(locs, 1.0, 0.1, 1.3, 0.0)
    C1 = dense.cov_matrix(locs, 1.0, 0.1, 1.3, 1e-3)
    assert np.array_equal(C0, C0.T)
    assert np.all(np.diag(C0) == 1.0)
    off = ~np.eye(300, dtype=bool)
    assert np.array_equal(C0[off], C1[off])
    assert np.allclose(np.diag(C1), 1.0 + 1e-3, rtol=0, atol=1e-15)
    assert np.linalg.eigvalsh(C1).min() > 0


def test_quad_equals_xi_norm_when_z_is_L_xi():
    # Z = L xi  =>  Z^T C^{-1} Z = ||xi||^2 exactly (same dense factor)
    locs, xi = workloads.uniform(2000, seed=0)
    z = dense.sample_field(locs, xi, 1.0, 0.1, 0.5, 1e-4)
    _, _, q = dense.loglik_parts(locs, z, 1.0, 0.1, 0.5, 1e-4)
    assert abs(q - float(xi @ xi)) < 1e-8 * float(xi @ xi)


def test_invariances_permutation_rigid_motion_scale():
    locs, xi = workloads.uniform(500, seed=5)
    th = (1.3, 0.12, 0.9, 1e-4)
    ll = dense.loglik(locs, xi, *th)
    p = np.random.default_rng(9).permutation(500)
    assert abs(dense.loglik(locs[p], xi[p], *th) - ll) < 1e-9 * abs(ll)
    a = 0.7
    R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    moved = locs @ R.T + np.array([3.0, -2.0])
    assert abs(dense.loglik(moved, xi, *th) - ll) < 1e-8 * abs(ll)
    c = 4.0
    assert abs(dense.loglik(c * locs, xi, th[0], c * th[1], th[2], th[3]) - ll) < 1e-8 * abs(ll)


# ---------------------------------------------------------------- 1-D Markov pins

def test_dense_matches_ou_closed_form():
    locs, xi = workloads.line(600, seed=4)
    z = xi * 0.8
    ll, ld, q = dense.loglik_parts(locs, z, 1.4, 0.05, 0.5, 0.0)
    llo, ldo, qo = markov.ou_loglik(locs[:, 0], z, 1.4, 0.05)
    assert abs(ld - ldo) < 1e-9 * abs(ldo)
    assert abs(q - qo) < 1e-9 * abs(qo)
    assert abs(ll - llo) < 1e-9 * abs(llo)


@pytest.mark.parametrize("nu,tau2,ell", [(0.5, 0.0, 0.03), (0.5, 1e-3, 0.03),
                                         (1.5, 0.0, 0.002), (1.5, 1e-4, 0.03)])
def test_dense_matches_kalman(nu, tau2, ell):
    # (nu = 3/2 without nugget needs a short range to stay well conditioned)
    locs, xi = workloads.line(500, seed=6)
    z = xi
    ll, ld, q = dense.loglik_parts(locs, z, 0.9, ell, nu, tau2)
    llk, ldk, qk = markov.kalman_loglik(locs[:, 0], z, 0.9, ell, nu, tau2)
    assert abs(ll - llk) < 1e-8 * max(abs(llk), 1.0)
    assert abs(ld - ldk) < 1e-8 * max(abs(ldk), 1.0)


def test_ou_closed_form_matches_kalman():
    locs, xi = workloads.line(2000, seed=8)
    a = markov.ou_loglik(locs[:, 0], xi, 1.0, 0.01)
    b = markov.kalman_loglik(locs[:, 0], xi, 1.0, 0.01, 0.5, 0.0)
    assert abs(a[0] - b[0]) < 1e-9 * abs(a[0])


def test_config1_anchor():
    # configuration with n=2000 uniform points (seed 0), theta = (1, 0.1, 0.5),
    # nugget 1e-4, Z = L xi: the dense FP64 values every H-path result is
    # compared with.  Independent of the oracle: q must equal ||xi||^2.
    locs, xi = workloads.uniform(2000, seed=0)
    z = dense.sample_field(locs, xi, 1.0, 0.1, 0.5, 1e-4)
    ll, ld, q = dense.loglik_parts(locs, z, 1.0, 0.1, 0.5, 1e-4)
    assert abs(q - float(xi @ xi)) < 1e-8 * q
    n = 2000
    assert abs(ll - (-0.5 * n * math.log(2 * math.pi) - 0.5 * ld - 0.5 * q)) < 1e-9


# ---------------------------------------------------------------- dense.solve
def test_dense_solve_two_points_closed_form():
    # n = 2: C = [[a, b], [b, a]] with a = sigma^2 + tau^2, b = C(h); its
    # inverse is [[a, -b], [-b, a]] / (a^2 - b^2)
    locs = np.array([[0.1, 0.2], [0.4, 0.6]])
    s2, ell, nu, tau2 = 1.3, 0.2, 0.5, 0.05
    b = s2 * math.exp(-0.5 / ell)            # h = 0.5, exponential kernel (nu = 1/2)
    a = s2 + tau2
    z = np.array([0.7, -1.1])
    want = np.array([a * z[0] - b * z[1], -b * z[0] + a * z[1]]) / (a * a - b * b)
    np.testing.assert_allclose(dense.solve(locs, z, s2, ell, nu, tau2), want, rtol=1e-14)


def test_dense_solve_residual_and_quadratic_form():
    # x = C^{-1} z solves C x = z (residual at rounding level for a well
    # conditioned C) and z^T x is the quadratic form of Eq. (1)
    locs, xi = workloads.uniform(400, seed=4)
    th = (1.1, 0.07, 1.3, 1e-2)
    x = dense.solve(locs, xi, *th)
    C = dense.cov_matrix(locs, *th)
    assert np.linalg.norm(C @ x - xi) <= 1e-12 * np.linalg.norm(C, 2) * np.linalg.norm(x)
    _, _, q = dense.loglik_parts(locs, xi, *th)
    assert abs(float(xi @ x) - q) <= 1e-10 * q


# ---------------------------------------------------------------- config-1 anchor
def test_config1_anchor_values():
    # n = 2000 locations U([0,1]^2) and xi from default_rng(0) (locations first),
    # Z = L xi with the exact factor; theta = (1, 0.1, 0.5), nugget 1e-4.  The
    # values were computed independently (dense FP64 with LAPACK, outside this
    # oracle) when the workloads were specified: logdet -3388.72409326966,
    # q 1968.12766144384, L -1127.57885049644.
    locs, xi = workloads.uniform(2000, seed=0)
    th = (1.0, 0.1, 0.5, 1e-4)
    z = dense.sample_field(locs, xi, *th)
    ll, ld, q = dense.loglik_parts(locs, z, *th)
    assert abs(ld - (-3388.72409326966)) < 2e-9 * 3388.7
    assert abs(q - 1968.12766144384) < 2e-9 * 1968.1
    assert abs(ll - (-1127.57885049644)) < 2e-9 * 1127.6
    # and q = ||xi||^2 exactly up to rounding when Z = L xi
    assert abs(q - float(xi @ xi)) < 1e-9 * q


def test_cov_block_tiles_cov_matrix():
    # the block assembly used for the large dense fixtures is the same
    # arithmetic as cov_matrix, entry for entry
    locs, _ = workloads.uniform(300, seed=8)
    th = (1.2, 0.09, 0.8)
    C = dense.cov_matrix(locs, *th, 0.0)
    B = np.vstack([dense.cov_block(locs[i:i + 64], locs, *th) for i in range(0, 300, 64)])
    assert np.array_equal(B, C)


def test_torch_lapack_path_matches_scipy():
    # the MKL route used for the n = 32768 fixtures against the SciPy route
    locs, xi = workloads.uniform(500, seed=9)
    C = dense.cov_matrix(locs, 1.0, 0.1, 0.8, 1e-4)
    L1 = dense.cholesky_lapack(C)
    L2 = dense.cholesky_torch(C)
    assert np.max(np.abs(L1 - L2)) < 1e-12 * np.max(np.abs(L1))
    v1 = dense.forward_solve_lapack(L1, xi)
    v2 = dense.forward_solve_torch(L2, xi)
    assert np.max(np.abs(v1 - v2)) < 1e-9 * np.max(np.abs(v1))
