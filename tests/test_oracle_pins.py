"""Pins for the CPU oracle: each test ties a piece of the oracle to something
other than itself -- closed forms, library routines, geometric identities,
the printed Appendix-B Jacobian, limits and invariants.  CPU only."""
import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import CubicSpline

from oracle import Problem, flat_state, residual, rule_weights, weights
from oracle import linear as L
from oracle import equations as R
from oracle.solve import gmres, jvp_complex, jvp_fd, newton

C1 = Problem(31, 11, -8.0, 8.0, 8.0, F=0.7, eps=0.05)
TINY = Problem(9, 5, -3.0, 3.0, 2.0, F=0.7, eps=0.3)
SMALL = Problem(15, 7, -6.0, 6.0, 5.0, F=0.7, eps=0.05)


def _noisy(prob, scale, seed):
    rng = np.random.default_rng(seed)
    return flat_state(prob) + scale * rng.standard_normal(prob.n_unknowns)


# --- whole residual -------------------------------------------------------
@pytest.mark.parametrize("prob", [
    C1.with_(eps=0.0),
    C1.with_(eps=0.0, weights="simpson"),
    C1.with_(eps=0.0, spline_bc="notaknot"),
    Problem(181, 61, -16.0, 8.0, 12.0, F=0.7, eps=0.0),
])
def test_flat_state_zero_source_gives_exact_zero(prob):
    """eps = 0 and a flat surface (phi = x): every term vanishes exactly."""
    E = residual(prob, flat_state(prob))
    assert np.all(E == 0.0)


def test_flat_state_with_source_only_E2_nonzero():
    E = residual(C1, flat_state(C1))
    NM = C1.N * C1.M
    assert np.all(E[:NM] == 0.0)
    E2 = E[NM:].reshape(C1.M, C1.N)
    assert np.all(E2[:, 0] == 0.0)
    xs, ys = C1.xs(), C1.y()
    np.testing.assert_allclose(E2[:, 1:], C1.eps / np.sqrt(xs[None] ** 2 + ys[:, None] ** 2 + 1),
                               rtol=1e-15, atol=0)


# --- a2 trapezoid scan ------------------------------------------------------
def test_trapezoid_exact_on_linear_slopes_and_radiation_rows():
    prob = C1
    x = prob.x()
    a, b = 0.3, -0.02
    fx = np.tile(a + b * x, (prob.M, 1))
    f1 = np.full(prob.M, 1.7)
    f = R.trapezoid_rows(fx, f1, prob.dx)
    exact = 1.7 + a * (x - x[0]) + 0.5 * b * (x ** 2 - x[0] ** 2)
    np.testing.assert_allclose(f, np.tile(exact, (prob.M, 1)), rtol=0, atol=1e-13)
    # E3 and E5 hold identically after eliminating phi_1, zeta_1
    u = _noisy(prob, 1e-3, 3)
    psix, zetax = R.unpack(prob, u)
    psi1 = (-prob.x1 / prob.nu) * psix[:, 0]
    E3 = prob.x1 * psix[:, 0] + prob.nu * psi1
    np.testing.assert_allclose(E3, 0.0, atol=1e-15)


# --- a3 spline -------------------------------------------------------------
def test_spline_reproduces_cubic_with_zero_slope_at_centreline():
    y = np.arange(9) * 0.4
    f = 1.0 + y ** 2 + y ** 3
    s = R.spline_slopes(np.stack([f, 2 * f], axis=1), 0.4, "clamped0")
    np.testing.assert_allclose(s[:, 0], 2 * y + 3 * y ** 2, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(s[:, 1], 2 * (2 * y + 3 * y ** 2), rtol=1e-13, atol=1e-13)


def test_spline_notaknot_reproduces_any_cubic():
    y = np.arange(7) * 0.3
    f = 2.0 - y + 0.5 * y ** 2 - 0.7 * y ** 3
    s = R.spline_slopes(f[:, None], 0.3, "notaknot")[:, 0]
    np.testing.assert_allclose(s, -1 + y - 2.1 * y ** 2, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("bc,scipy_bc", [("clamped0", ((1, np.zeros(5)), "not-a-knot")),
                                         ("notaknot", "not-a-knot")])
def test_spline_matches_scipy_cubicspline(bc, scipy_bc):
    rng = np.random.default_rng(7)
    h = 0.25
    y = np.arange(13) * h
    f = rng.standard_normal((13, 5))
    s = R.spline_slopes(f, h, bc)
    ref = CubicSpline(y, f, axis=0, bc_type=scipy_bc).derivative()(y)
    np.testing.assert_allclose(s, ref, rtol=1e-12, atol=1e-12)


# --- a4 closed form of I ------------------------------------------------------
def _G_polar(A, B, C, a, b):
    """G(a,b) in polar coordinates about the corner: the radial integral of r/r
    is the distance to the far edge, min(a/cos t, b/sin t)."""
    def q(t):
        c, s = np.cos(t), np.sin(t)
        return np.sqrt(A * c * c + B * c * s + C * s * s)
    tc = np.arctan2(b, a)
    g1 = integrate.quad(lambda t: a / np.cos(t) / q(t), 0, tc, epsabs=0, epsrel=2e-14, limit=200)[0]
    g2 = integrate.quad(lambda t: b / np.sin(t) / q(t), tc, np.pi / 2, epsabs=0, epsrel=2e-14,
                        limit=200)[0]
    return g1 + g2


@pytest.mark.parametrize("seed", range(6))
def test_G_closed_form_matches_polar_quadrature(seed):
    rng = np.random.default_rng(seed)
    zx, zy = rng.normal(0, 1.5, 2)
    A, B, C = 1 + zx ** 2, 2 * zx * zy, 1 + zy ** 2
    for sgn in (1.0, -1.0):
        for a, b in [(0.3, 7.0), (5.0, 0.02), (1.0, 1.0), (12.0, 3.3)]:
            got = R.G_rect(A, sgn * B, C, a, b)
            ref = _G_polar(A, sgn * B, C, a, b)
            assert abs(got - ref) <= 1e-12 * abs(ref), (a, b, got, ref)
            assert got > 0


def test_G_reduces_to_asinh_for_the_isotropic_form():
    for a, b in [(0.1, 3.0), (2.0, 2.0), (7.5, 0.4)]:
        ref = a * np.arcsinh(b / a) + b * np.arcsinh(a / b)
        assert abs(R.G_rect(1.0, 0.0, 1.0, a, b) - ref) <= 1e-14 * ref


def test_G_zero_on_degenerate_rectangles():
    assert R.G_rect(1.3, 0.2, 1.1, 0.0, 2.0) == 0.0
    assert R.G_rect(1.3, 0.2, 1.1, 2.0, 0.0) == 0.0


def test_I_with_images_matches_quadrature_over_the_rectangle():
    """Direct part: polar quadrature of each quadrant about (x*, y*).  Image part:
    plain 2-D adaptive quadrature (smooth for y* > 0)."""
    x1, xN, yM = -4.0, 3.0, 2.5
    zx, zy = 0.4, -0.7
    A, B, C = 1 + zx ** 2, 2 * zx * zy, 1 + zy ** 2
    xs, ys = 0.35, 0.8
    got = R.I_closed(A, B, C, xs - x1, xN - xs, ys, yM - ys, ys, yM, True)
    direct = (_G_polar(A, B, C, xN - xs, yM - ys) + _G_polar(A, -B, C, x1 * -1 + xs, yM - ys)
              + _G_polar(A, -B, C, xN - xs, ys) + _G_polar(A, B, C, xs - x1, ys))
    image = integrate.dblquad(
        lambda y, x: 1 / np.sqrt(A * (x - xs) ** 2 - B * (x - xs) * (y + ys) + C * (y + ys) ** 2),
        x1, xN, 0.0, yM, epsabs=1e-13, epsrel=1e-13)[0]
    assert abs(got - (direct + image)) <= 1e-10 * got


# --- weights ----------------------------------------------------------------
@pytest.mark.parametrize("rule", ["trapezoid", "simpson"])
def test_weights_integrate_exactly(rule):
    prob = C1.with_(weights=rule)
    w = weights(prob)
    area = (prob.xN - prob.x1) * prob.yM
    assert abs(w.sum() - area) <= 1e-12 * area
    X, Y = np.meshgrid(prob.x(), prob.y())
    if rule == "trapezoid":
        f = (1 + 2 * X) * (3 - Y)   # bilinear
        ex = ((prob.xN - prob.x1) + (prob.xN ** 2 - prob.x1 ** 2)) * (3 * prob.yM - prob.yM ** 2 / 2)
    else:
        f = (X + 9) ** 3 * Y ** 3   # bicubic
        ex = ((prob.xN + 9) ** 4 - (prob.x1 + 9) ** 4) / 4 * prob.yM ** 4 / 4
    assert abs((w * f).sum() - ex) <= 1e-11 * abs(ex)
    np.testing.assert_allclose(rule_weights(5, 1.0, "simpson"), [1 / 3, 4 / 3, 2 / 3, 4 / 3, 1 / 3])


# --- a5 kernels -------------------------------------------------------------
def test_K1_is_the_normal_derivative_of_the_greens_function():
    """K1 = -n_Q . grad_Q (1/|Q - P|) with n_Q = (-zeta_x, -zeta_y, 1) at the
    integration point Q, plus the same for the mirror point P' = (x*, -y*, zeta*).
    The gradient is taken by complex-step differentiation of 1/|Q - P|."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        xq, yq, zq, zxq, zyq = rng.normal(size=5)
        yq = abs(yq)
        xp, yp, zp = rng.normal(size=3)
        yp = abs(yp)
        nq = np.array([-zxq, -zyq, 1.0])

        def greens(P, Q):
            d = Q - P
            return 1.0 / np.sqrt(d @ d)

        def dn(P):
            Q = np.array([xq, yq, zq], dtype=complex)
            return -(greens(P, Q + 1j * 1e-30 * nq).imag / 1e-30)

        ref = dn(np.array([xp, yp, zp])) + dn(np.array([xp, -yp, zp]))
        K1, K2, _ = R.kernels(xq - xp, yq - yp, yq + yp, zq - zp, zxq, zyq, 1.0, 0.0, 1.0, True)
        assert abs(K1 - ref) <= 1e-13 * max(1.0, abs(ref))
        r1 = np.sqrt((xq - xp) ** 2 + (yq - yp) ** 2 + (zq - zp) ** 2)
        r2 = np.sqrt((xq - xp) ** 2 + (yq + yp) ** 2 + (zq - zp) ** 2)
        assert abs(K2 - (1 / r1 + 1 / r2)) <= 1e-14 * K2


def test_S2_equals_K2_on_a_plane_through_the_collocation_point():
    """S2 is K2 with zeta - zeta* replaced by its linear part, so on a plane
    zeta = zeta* + a dx (even in y: b = 0 keeps the mirror point on it) they agree."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        a = rng.normal()
        dx, dy = rng.normal(size=2)
        ys = abs(rng.normal())
        A, B, C = 1 + a * a, 0.0, 1.0
        _, K2, S2 = R.kernels(dx, dy, dy + 2 * ys, a * dx, a, 0.0, A, B, C, True)
        assert abs(K2 - S2) <= 1e-14 * K2
        b = rng.normal()
        _, K2, S2 = R.kernels(dx, dy, dy + 2 * ys, a * dx + b * dy, a, b, 1 + a * a, 2 * a * b,
                              1 + b * b, False)
        assert abs(K2 - S2) <= 1e-14 * K2


# --- images: half domain == full domain ------------------------------------------
@pytest.mark.parametrize("rule", ["trapezoid", "simpson"])
def test_half_domain_with_images_equals_full_domain_without(rule):
    """Even extension of a half-domain state to y in [-y_M, y_M]: the full-plane
    discretisation (no images, not-a-knot spline ends) must give the same
    residual rows for y* >= 0.  Pins the image terms, the K1 image distance
    and the centreline spline condition."""
    prob = Problem(13, 7, -4.0, 4.0, 3.0, F=0.7, eps=0.4, weights=rule)
    rng = np.random.default_rng(2)
    u = flat_state(prob) + 0.05 * rng.standard_normal(prob.n_unknowns)
    psix, zetax = R.unpack(prob, u)
    E1h, E2h, E4h, E6h = R._residual_geom(prob, R._half_geom(prob), psix, zetax)
    E1f, E2f, E4f, E6f = R.residual_full_domain(prob, R.even_extension(psix),
                                                R.even_extension(zetax))
    M = prob.M
    np.testing.assert_allclose(E1f[M - 1:], E1h, rtol=0, atol=1e-12)
    np.testing.assert_allclose(E2f[M - 1:], E2h, rtol=0, atol=1e-11)
    np.testing.assert_allclose(E2f[:M], E2h[::-1], rtol=0, atol=1e-11)
    np.testing.assert_allclose(E4f[M - 1:], E4h, rtol=0, atol=1e-13)


def test_dropping_the_image_correction_breaks_the_symmetry_pin():
    """The pin above is sensitive: the printed (y - y*)^2 image denominator fails it."""
    prob = Problem(13, 7, -4.0, 4.0, 3.0, F=0.7, eps=0.4)
    rng = np.random.default_rng(2)
    u = flat_state(prob) + 0.05 * rng.standard_normal(prob.n_unknowns)
    psix, zetax = R.unpack(prob, u)
    orig = R.kernels

    def typo(dx, dy, dyp, dz, zx, zy, A, B, C, images):
        K1, K2, S2 = orig(dx, dy, dyp, dz, zx, zy, A, B, C, images)
        if images:
            n0 = dz - dx * zx
            good = (n0 - dyp * zy) / (dx * dx + dyp * dyp + dz * dz) ** 1.5
            bad = (n0 - dyp * zy) / (dx * dx + dy * dy + dz * dz) ** 1.5
            K1 = K1 - good + bad
        return K1, K2, S2

    R.kernels = typo
    try:
        _, E2h, _, _ = R._residual_geom(prob, R._half_geom(prob), psix, zetax)
    finally:
        R.kernels = orig
    _, E2f, _, _ = R.residual_full_domain(prob, R.even_extension(psix), R.even_extension(zetax))
    assert np.abs(E2f[prob.M - 1:] - E2h).max() > 1e-6


# --- E1 --------------------------------------------------------------------------
def test_bernoulli_rewrite_matches_velocity_components():
    """E1 is (1/2)|grad Phi|^2 + zeta/F^2 - 1/2 with Phi_x, Phi_y, Phi_z recovered
    from the surface derivatives: phi_x = Phi_x + Phi_z zeta_x,
    phi_y = Phi_y + Phi_z zeta_y and the kinematic condition
    Phi_z = Phi_x zeta_x + Phi_y zeta_y."""
    rng = np.random.default_rng(4)
    prob = TINY
    f = R.Fields(*([None] * 6), ps=None, pxs=rng.normal(0, .3, 8), pys=rng.normal(0, .3, 8),
                 zs=rng.normal(0, .1, 8), zxs=rng.normal(0, .5, 8), zys=rng.normal(0, .5, 8))
    E1 = R.bernoulli(prob, f)
    for i in range(8):
        px, py, zx, zy = 1 + f.pxs[i], f.pys[i], f.zxs[i], f.zys[i]
        M3 = np.array([[1, 0, zx], [0, 1, zy], [zx, zy, -1.0]])
        Vx, Vy, Vz = np.linalg.solve(M3, [px, py, 0.0])
        ref = 0.5 * (Vx * Vx + Vy * Vy + Vz * Vz) + f.zs[i] / prob.F ** 2 - 0.5
        assert abs(E1[i] - ref) <= 1e-14


# --- derivatives: J(u_flat) = J_lin + eps J_src -------------------------------
@pytest.mark.parametrize("rule", ["trapezoid", "simpson"])
def test_jacobian_at_flat_state_is_the_appendix_B_matrix(rule):
    prob = TINY.with_(weights=rule)
    u = flat_state(prob)
    n = u.size
    J = np.empty((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        J[:, i] = residual(prob, u + 1j * 1e-30 * e).imag / 1e-30
        e[i] = 0.0
    ref = L.jlin_dense(prob) + prob.eps * L.jsrc_dense(prob)
    assert np.abs(J - ref).max() <= 1e-13 * np.abs(ref).max()


def test_fd_jvp_converges_to_exact_jvp_linearly_in_h():
    prob = TINY
    u = _noisy(prob, 0.02, 8)
    z = np.random.default_rng(9).standard_normal(u.size)
    Eu = residual(prob, u)
    ex = jvp_complex(prob, u, z)
    errs = [np.abs(jvp_fd(prob, u, Eu, z, h) - ex).max() for h in (1e-3, 1e-4, 1e-5)]
    assert errs[0] / errs[1] == pytest.approx(10, rel=0.1)
    assert errs[1] / errs[2] == pytest.approx(10, rel=0.1)
    assert errs[2] <= 1e-2 * np.abs(ex).max()


# --- roots ----------------------------------------------------------------------
def test_small_source_limit_is_the_linear_solution():
    """u(eps) = u_flat + eps u1 + O(eps^2) with J_lin u1 = -s."""
    prob = SMALL
    u1 = L.linear_solution(prob.with_(eps=1.0)) - flat_state(prob)
    ratios = []
    for e in (0.02, 0.01, 0.005):
        p = prob.with_(eps=e)
        u, info = newton(p, flat_state(p), tol=1e-13)
        assert info.converged
        ratios.append(np.abs(u - flat_state(p) - e * u1).max() / e ** 2)
    assert ratios[0] > 0
    assert max(ratios) / min(ratios) < 1.3


def test_dense_newton_is_quadratic_and_agrees_with_jfnk():
    prob = SMALL
    ud, infod = newton(prob, flat_state(prob), tol=1e-12, linear="dense")
    assert infod.converged
    e = infod.norms
    assert e[2] <= 10 * e[1] ** 2 / e[0] + 1e-13
    uj, infoj = newton(prob, flat_state(prob), tol=1e-12)
    assert infoj.converged
    assert np.abs(ud - uj).max() <= 1e-10


def test_31x11_root_satisfies_invariants():
    u, info = newton(C1, flat_state(C1), tol=1e-12)
    assert info.converged
    parts = R.residual_parts(C1, u)
    assert np.abs(parts["E4"]).max() <= 1e-12 and np.abs(parts["E6"]).max() <= 1e-12
    assert parts["fields"].zs.max() <= C1.F ** 2 / 2


# --- preconditioner (Appendix C) ---------------------------------------------------
def test_three_step_solve_equals_dense_solve():
    prob = TINY
    rng = np.random.default_rng(3)
    b = rng.standard_normal(prob.n_unknowns)
    for q in (0, 1, prob.M - 1):
        pre = L.BlockPreconditioner(prob, q)
        P = pre.matrix()
        x = pre.solve(b)
        np.testing.assert_allclose(P @ x, b, rtol=0, atol=1e-10 * np.abs(b).max())
    pre = L.BlockPreconditioner(prob, prob.M - 1)
    np.testing.assert_array_equal(pre.matrix(), L.jlin_dense(prob))


def test_full_linear_preconditioner_solves_linear_problem_in_one_iteration():
    prob = SMALL
    pre = L.BlockPreconditioner(prob, prob.M - 1)
    J = L.jlin_dense(prob)
    b = -prob.eps * L.source_vector(prob)
    v = np.random.default_rng(1).standard_normal(prob.n_unknowns)
    np.testing.assert_allclose(pre.solve(J @ v), v, rtol=0, atol=1e-9 * np.abs(v).max())
    x, its, res = gmres(lambda y: J @ y, b, pre.solve, tol=1e-10 * np.linalg.norm(b))
    assert its == 1


@pytest.mark.parametrize("q", [0, 2, 6])
@pytest.mark.parametrize("rule", ["trapezoid", "simpson"])
def test_row_wise_p_times_x_equals_the_dense_preconditioner(q, rule):
    """p_rows forms entries of P x from the blocks without a dense P (for meshes whose P
    does not fit); on every row of a small mesh it must equal BlockPreconditioner's
    dense matrix times x, and with absolute=True |P| |x|.  K3_sum_at must equal the
    sums that the dense D uses."""
    prob = C1.with_(weights=rule)
    Pm = L.BlockPreconditioner(prob, q).matrix()
    x = np.random.default_rng(q).standard_normal(prob.n_unknowns)
    rows = np.arange(prob.n_unknowns)
    y = L.p_rows(prob, q, rows, x)
    ya = L.p_rows(prob, q, rows, x, absolute=True)
    scale = np.abs(Pm) @ np.abs(x)
    assert np.abs(y - Pm @ x).max() <= 1e-14 * scale.max()
    assert np.abs(ya - scale).max() <= 1e-14 * scale.max()
    S = L.K3_sums(prob)
    for l in (0, 3, prob.M - 1):
        for k in (0, 7, prob.N - 2):
            assert abs(L.K3_sum_at(prob, l, k) - S[l, k]) <= 1e-14 * abs(S[l, k])
