"""Plain FP64 CPU oracle for the nonlinear residual E(u).

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

Every function works on real float64 arrays and also on complex128 arrays, so
that complex-step differentiation (Im E(u + i h z) / h) gives an exact
directional derivative of the same discrete system.  For that reason nothing
here uses abs(), max() or a comparison on a value that depends on u, except
for branch choices taken on the real part where both branches are the same
analytic function.

Reduced unknowns.  The paper's vector u has 2(N+1)M entries (eq. unknowns):
phi_{1,l}, (phi_x)_{1..N,l} for each row, then the same for zeta.  The first
and third radiation equations (eq. numUpRadiation; E3 and E5 in Appendix A)
are linear and explicit in phi_{1,l} and zeta_{1,l}:
    phi_{1,l} - x_1 = -(x_1/nu) ((phi_x)_{1,l} - 1),   zeta_{1,l} = -(x_1/nu) (zeta_x)_{1,l},
so those 2M unknowns and equations are eliminated.  The reduced vector is
    u = [ (phi_x)_{1..N,1}, ..., (phi_x)_{1..N,M},  (zeta_x)_{1..N,1}, ..., (zeta_x)_{1..N,M} ]
(2NM entries, x fastest) and the reduced residual, ordered as Appendix A with
E3/E5 removed, is
    E = [ E4_l, E1_{1..N-1,l} ]_{l=1..M}  followed by  [ E6_l, E2_{1..N-1,l} ]_{l=1..M}.

The perturbation potential psi = phi - x is carried instead of phi: the
integrand of the boundary-integral equation (eq. IntegroEqn) contains exactly
phi - phi* - x + x* = psi - psi*, and the radiation rows are written in
phi - x and phi_x - 1.  This is the same discrete system.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .problem import Problem, rule_weights

TWO_PI = 2.0 * np.pi


# ---------------------------------------------------------------------------
# Steps a1-a3: unknowns -> grid fields
# ---------------------------------------------------------------------------
def unpack(prob: Problem, u):
    """u (2NM) -> psi_x, zeta_x as (M, N) arrays.  psi_x = phi_x - 1."""
    N, M = prob.N, prob.M
    NM = N * M
    u = np.asarray(u)
    if u.shape != (2 * NM,):
        raise ValueError(f"u must have length {2 * NM}")
    psix = (u[:NM] - 1.0).reshape(M, N)
    zetax = u[NM:].reshape(M, N)
    return psix, zetax


def trapezoid_rows(fx, f1, dx: float):
    """Trapezoidal-rule integration along x for every row (eq. zetaapprox):
    f_{k+1} = f_k + dx/2 (fx_k + fx_{k+1}), starting from f_1."""
    f = np.empty_like(fx)
    f[:, 0] = f1
    for k in range(fx.shape[1] - 1):
        f[:, k + 1] = f[:, k] + 0.5 * dx * (fx[:, k] + fx[:, k + 1])
    return f


def spline_slopes(f, h: float, bc: str):
    """Slopes at the knots of the interpolating cubic spline through the
    columns of f (rows = equally spaced knots y_1..y_R, spacing h).

    The paper fits a cubic spline through zeta_{k,1..M} for each k (numerical
    discretisation section) but does not state its end conditions.  Reading:
      bc == "clamped0": slope 0 at the first knot (y = 0: zeta and phi are even
                        in y) and not-a-knot at the last knot;
      bc == "notaknot": not-a-knot at both ends.
    Interior knots: continuity of the second derivative of the piecewise
    cubic Hermite interpolant gives s_{j-1} + 4 s_j + s_{j+1} = 3 (f_{j+1} - f_{j-1}) / h.
    Not-a-knot at knot 2 (third derivative continuous there):
      s_1 - s_3 = 2 (d_1 - d_2) / h with d_j = f_{j+1} - f_j,
    and symmetrically at the far end.  The system is solved densely.
    """
    R = f.shape[0]
    if R < 4:
        raise ValueError("spline needs at least 4 knots")
    Mat = np.zeros((R, R))
    rhs = np.zeros(f.shape, dtype=np.result_type(f, 1.0))
    for j in range(1, R - 1):
        Mat[j, j - 1] = 1.0
        Mat[j, j] = 4.0
        Mat[j, j + 1] = 1.0
        rhs[j] = 3.0 * (f[j + 1] - f[j - 1]) / h
    d = f[1:] - f[:-1]
    if bc == "clamped0":
        Mat[0, 0] = 1.0
        rhs[0] = 0.0
    elif bc == "notaknot":
        Mat[0, 0] = 1.0
        Mat[0, 2] = -1.0
        rhs[0] = 2.0 * (d[0] - d[1]) / h
    else:
        raise ValueError(bc)
    Mat[R - 1, R - 3] = 1.0
    Mat[R - 1, R - 1] = -1.0
    rhs[R - 1] = 2.0 * (d[R - 3] - d[R - 2]) / h
    return np.linalg.solve(Mat, rhs)


# ---------------------------------------------------------------------------
# Step a4: the closed form of I (eq. IS2)
# ---------------------------------------------------------------------------
def _Lint(P, B, R, tau):
    """L(P,B,R;tau) = integral_0^tau dt / sqrt(P t^2 + B t + R), P > 0, 4PR > B^2.

    Antiderivative: P^{-1/2} ln(2 sqrt(P) sqrt(P t^2 + B t + R) + 2 P t + B).
    Where 2Pt + B < 0 the argument is rewritten with its conjugate,
    (4PR - B^2) / (2 sqrt(P) sqrt(...) - 2Pt - B), which is the same number
    without cancellation."""
    sP = np.sqrt(P)
    q = np.sqrt(P * tau * tau + B * tau + R)
    disc = 4.0 * P * R - B * B
    lin = 2.0 * P * tau + B
    top = np.where(np.real(lin) >= 0.0, 2.0 * sP * q + lin, disc / (2.0 * sP * q - lin))
    s0 = 2.0 * np.sqrt(P * R)
    bot = np.where(np.real(B) >= 0.0, s0 + B, disc / (s0 - B))
    return (np.log(top) - np.log(bot)) / sP


def G_rect(A, B, C, a, b):
    """G(a,b) = integral_0^a integral_0^b dY dX / sqrt(A X^2 + B X Y + C Y^2), a, b >= 0.

    Split the rectangle on its diagonal.  Below it substitute Y = t X
    (t in [0, b/a]); above it X = s Y (s in [0, a/b]):
        G = a L(C,B,A; b/a) + b L(A,B,C; a/b),    G = 0 if a = 0 or b = 0.
    """
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    ok = (a > 0.0) & (b > 0.0)
    sa = np.where(ok, a, 1.0)
    sb = np.where(ok, b, 1.0)
    val = sa * _Lint(C, B, A, sb / sa) + sb * _Lint(A, B, C, sa / sb)
    return np.where(ok, val, 0.0)


def I_closed(A, B, C, a1, a2, b1, b2, ystar, ytop, images: bool):
    """I = integral over the truncated rectangle of S2 (eq. IS2), in closed form.

    With X = x - x*, Y = y - y*, the direct part of S2 is 1/sqrt(AX^2 + BXY + CY^2)
    over X in [-a1, a2], Y in [-b1, b2]; splitting at X = 0 and Y = 0 and
    reflecting each quadrant onto X, Y >= 0 flips the sign of B in the two
    mixed quadrants.  The image part is 1/sqrt(AX^2 - BXY' + CY'^2) with
    Y' = y + y* in [y*, y_M + y*] (only on the half domain, y_1 = 0).
    """
    direct = (G_rect(A, B, C, a2, b2) + G_rect(A, -B, C, a1, b2)
              + G_rect(A, -B, C, a2, b1) + G_rect(A, B, C, a1, b1))
    if not images:
        return direct
    image = (G_rect(A, -B, C, a2, ytop + ystar) + G_rect(A, B, C, a1, ytop + ystar)
             - G_rect(A, -B, C, a2, ystar) - G_rect(A, B, C, a1, ystar))
    return direct + image


# ---------------------------------------------------------------------------
# Step a5: kernel functions (eq. IntegroEqn, eq. S2)
# ---------------------------------------------------------------------------
def kernels(dx, dy, dyp, dz, zx, zy, A, B, C, images: bool):
    """K1, K2 and S2 at one (integration point, collocation point) pair.

    dx = x - x*, dy = y - y*, dyp = y + y*, dz = zeta(x,y) - zeta*;
    zx, zy are the surface slopes at the integration point (x, y);
    A, B, C belong to the collocation point.

    K1 is the normal derivative of the Green's function 1/R with the surface
    normal (-zeta_x, -zeta_y, 1) at the integration point.  Its image term is
    evaluated at the mirror point (x*, -y*, zeta*), whose distance has
    (y + y*)^2; the printed image denominator shows (y - y*)^2, which is a
    typesetting slip (the K2 image term has (y + y*)^2).
    """
    n0 = dz - dx * zx
    r1sq = dx * dx + dy * dy + dz * dz
    r1 = np.sqrt(r1sq)
    K1 = (n0 - dy * zy) / (r1sq * r1)
    K2 = 1.0 / r1
    S2 = 1.0 / np.sqrt(A * dx * dx + B * dx * dy + C * dy * dy)
    if images:
        r2sq = dx * dx + dyp * dyp + dz * dz
        r2 = np.sqrt(r2sq)
        K1 = K1 + (n0 - dyp * zy) / (r2sq * r2)
        K2 = K2 + 1.0 / r2
        S2 = S2 + 1.0 / np.sqrt(A * dx * dx - B * dx * dyp + C * dyp * dyp)
    return K1, K2, S2


# ---------------------------------------------------------------------------
# Geometry shared by the half-domain (images) and full-domain (no images) forms
# ---------------------------------------------------------------------------
@dataclass
class _Geom:
    N: int
    R: int              # number of rows
    x1: float
    xN: float
    dx: float
    dy: float
    yidx: np.ndarray    # integer row offsets: y_j = yidx[j] * dy
    wx: np.ndarray
    wy: np.ndarray
    ylo: float
    yhi: float
    images: bool
    bc: str

    @property
    def y(self):
        return self.yidx * self.dy


def _half_geom(prob: Problem) -> _Geom:
    return _Geom(prob.N, prob.M, prob.x1, prob.xN, prob.dx, prob.dy,
                 np.arange(prob.M), rule_weights(prob.N, prob.dx, prob.weights),
                 rule_weights(prob.M, prob.dy, prob.weights), 0.0, prob.yM, True,
                 prob.spline_bc)


def _full_geom(prob: Problem) -> _Geom:
    """The whole strip y in [-y_M, y_M] with 2M-1 rows and no image terms."""
    R = 2 * prob.M - 1
    return _Geom(prob.N, R, prob.x1, prob.xN, prob.dx, prob.dy,
                 np.arange(R) - (prob.M - 1), rule_weights(prob.N, prob.dx, prob.weights),
                 rule_weights(R, prob.dy, prob.weights), -prob.yM, prob.yM, False,
                 "notaknot")


@dataclass
class Fields:
    """Grid fields (R, N) and half-mesh fields (R, N-1) of one state."""
    psix: np.ndarray
    zetax: np.ndarray
    psi: np.ndarray
    zeta: np.ndarray
    psiy: np.ndarray
    zetay: np.ndarray
    ps: np.ndarray      # psi*
    pxs: np.ndarray     # psi_x*
    pys: np.ndarray     # psi_y*
    zs: np.ndarray      # zeta*
    zxs: np.ndarray     # zeta_x*
    zys: np.ndarray     # zeta_y*


def grid_fields(prob: Problem, geom: _Geom, psix, zetax) -> Fields:
    """Steps a1-a3 plus the two-point interpolation onto the half mesh."""
    c = -prob.x1 / prob.nu
    psi = trapezoid_rows(psix, c * psix[:, 0], geom.dx)
    zeta = trapezoid_rows(zetax, c * zetax[:, 0], geom.dx)
    psiy = spline_slopes(psi, geom.dy, geom.bc)
    zetay = spline_slopes(zeta, geom.dy, geom.bc)

    def half(f):
        return 0.5 * (f[:, :-1] + f[:, 1:])

    return Fields(psix, zetax, psi, zeta, psiy, zetay, half(psi), half(psix), half(psiy),
                  half(zeta), half(zetax), half(zetay))


def bernoulli(prob: Problem, f: Fields):
    """E1 at the half-mesh points (eq. freeSurfCond), phi_x* = 1 + psi_x*, phi_y* = psi_y*."""
    px = 1.0 + f.pxs
    py = f.pys
    zx, zy = f.zxs, f.zys
    num = (1.0 + zx * zx) * py * py + (1.0 + zy * zy) * px * px - 2.0 * zx * zy * px * py
    return 0.5 * num / (1.0 + zx * zx + zy * zy) + f.zs / (prob.F * prob.F) - 0.5


def pair_sum(geom: _Geom, f: Fields, *, block: int = 64, want_abs: bool = False, cols=None):
    """Sigma_{k,l} = sum_{i,j} w(i,j) [ (psi_ij - psi*) K1 + zeta_x,ij K2 - zeta_x* S2 ].

    The sum over every grid point (i,j) of the truncated domain for every
    collocation point (k,l), trapezoid (or Simpson) weights, the singular
    part zeta_x* S2 subtracted (numerical discretisation section).
    Offsets come from integers: x_i - x*_k = (i - k - 1/2) dx,
    y_j - y*_l = (j - l) dy and y_j + y*_l = (j + l) dy (row offsets).
    Returns (Sigma, sum of |terms| per part) when want_abs.  With cols (flat
    collocation indices l*(N-1) + k) only those points are summed; the rest
    of the returned array is NaN.
    """
    N, R = geom.N, geom.R
    Nc = N - 1
    w = (geom.wy[:, None] * geom.wx[None, :]).ravel()
    si = np.tile(np.arange(N), R)
    sj = np.repeat(geom.yidx, N)
    psi = f.psi.ravel()
    zeta = f.zeta.ravel()
    zx = f.zetax.ravel()
    zy = f.zetay.ravel()
    ck = np.tile(np.arange(Nc), R)
    cl = np.repeat(geom.yidx, Nc)
    ps = f.ps.ravel()
    zs = f.zs.ravel()
    zxs = f.zxs.ravel()
    zys = f.zys.ravel()
    A = 1.0 + zxs * zxs
    B = 2.0 * zxs * zys
    C = 1.0 + zys * zys
    out = np.full(Nc * R, np.nan, dtype=np.result_type(psi, zeta, zx, zy))
    mags = np.full((3, Nc * R), np.nan) if want_abs else None
    todo = np.arange(Nc * R) if cols is None else np.asarray(cols, dtype=np.int64)
    for p0 in range(0, todo.size, block):
        sl = todo[p0:p0 + block]
        dx = (si[None, :] - ck[sl, None] - 0.5) * geom.dx
        dy = (sj[None, :] - cl[sl, None]) * geom.dy
        dyp = (sj[None, :] + cl[sl, None]) * geom.dy
        dz = zeta[None, :] - zs[sl, None]
        K1, K2, S2 = kernels(dx, dy, dyp, dz, zx[None, :], zy[None, :],
                             A[sl, None], B[sl, None], C[sl, None], geom.images)
        t1 = w[None, :] * (psi[None, :] - ps[sl, None]) * K1
        t2 = w[None, :] * zx[None, :] * K2
        t3 = w[None, :] * zxs[sl, None] * S2
        out[sl] = (t1 + t2 - t3).sum(axis=1)
        if want_abs:
            mags[0, sl] = np.abs(t1).sum(axis=1)
            mags[1, sl] = np.abs(t2).sum(axis=1)
            mags[2, sl] = np.abs(t3).sum(axis=1)
    if want_abs:
        return out.reshape(R, Nc), mags.reshape(3, R, Nc)
    return out.reshape(R, Nc)


def _I_field(geom: _Geom, f: Fields):
    xs = geom.x1 + (np.arange(geom.N - 1) + 0.5) * geom.dx
    ys = geom.y
    A = 1.0 + f.zxs * f.zxs
    B = 2.0 * f.zxs * f.zys
    C = 1.0 + f.zys * f.zys
    a1 = np.broadcast_to(xs - geom.x1, A.shape)
    a2 = np.broadcast_to(geom.xN - xs, A.shape)
    ystar = np.broadcast_to(ys[:, None], A.shape)
    b1 = ystar - geom.ylo
    b2 = geom.yhi - ystar
    return I_closed(A, B, C, a1, a2, b1, b2, ystar, geom.yhi, geom.images)


def _residual_geom(prob: Problem, geom: _Geom, psix, zetax, want_parts=False, cols=None):
    f = grid_fields(prob, geom, psix, zetax)
    E1 = bernoulli(prob, f)
    xs = geom.x1 + (np.arange(geom.N - 1) + 0.5) * geom.dx
    ys = geom.y
    src = prob.eps / np.sqrt(xs[None, :] ** 2 + ys[:, None] ** 2 + (f.zs + 1.0) ** 2)
    I = _I_field(geom, f)
    if want_parts:
        Sig, mags = pair_sum(geom, f, want_abs=True, cols=cols)
    else:
        Sig = pair_sum(geom, f, cols=cols)
    E2 = TWO_PI * f.ps + src - Sig - f.zxs * I
    x1, dx, nu = prob.x1, geom.dx, prob.nu
    E4 = x1 * (psix[:, 1] - psix[:, 0]) / dx + nu * psix[:, 0]
    E6 = x1 * (zetax[:, 1] - zetax[:, 0]) / dx + nu * zetax[:, 0]
    if want_parts:
        return dict(fields=f, E1=E1, E2=E2, E4=E4, E6=E6, I=I, src=src, Sigma=Sig, mags=mags)
    return E1, E2, E4, E6


def pack(E1, E2, E4, E6):
    """Reduced Appendix-A order: [E4_l, E1_{.,l}]_l then [E6_l, E2_{.,l}]_l."""
    top = np.concatenate([E4[:, None], E1], axis=1).ravel()
    bot = np.concatenate([E6[:, None], E2], axis=1).ravel()
    return np.concatenate([top, bot])


def residual(prob: Problem, u):
    """E(u) for the half domain with image terms (steps a1-a6), reduced form."""
    psix, zetax = unpack(prob, u)
    E1, E2, E4, E6 = _residual_geom(prob, _half_geom(prob), psix, zetax)
    return pack(E1, E2, E4, E6)


def residual_parts(prob: Problem, u, cols=None):
    """Residual plus intermediate fields and per-row magnitudes (real u only)."""
    psix, zetax = unpack(prob, u)
    return _residual_geom(prob, _half_geom(prob), psix, zetax, want_parts=True, cols=cols)


def e2_index_to_col(prob: Problem, idx):
    """Index into E (must be an E2 entry) -> flat collocation index l*(N-1) + k."""
    idx = np.asarray(idx) - prob.N * prob.M
    l, r = np.divmod(idx, prob.N)
    if np.any(idx < 0) or np.any(r == 0):
        raise ValueError("not an E2 entry")
    return l * (prob.N - 1) + (r - 1)


def residual_rows(prob: Problem, u, rows):
    """E(u)[rows] and row_scale(u)[rows], computing the all-pairs sum only at the
    collocation points that the requested E2 entries need."""
    rows = np.asarray(rows)
    NM = prob.N * prob.M
    e2 = rows[(rows >= NM) & ((rows - NM) % prob.N != 0)]
    cols = e2_index_to_col(prob, e2) if e2.size else np.zeros(0, dtype=np.int64)
    parts = residual_parts(prob, u, cols=cols)
    E = pack(parts["E1"], parts["E2"], parts["E4"], parts["E6"])
    return E[rows], _scale_from_parts(prob, parts)[rows]


def row_scale(prob: Problem, u):
    """Per-equation magnitude: the sum of the absolute values of the terms that
    make up each residual entry, floored at 1.  A parity tolerance relative to
    this scale measures rounding against the size of what was summed."""
    return _scale_from_parts(prob, residual_parts(prob, u))


def _scale_from_parts(prob: Problem, parts):
    f = parts["fields"]
    mags = parts["mags"]
    s2 = (mags.sum(axis=0) + np.abs(f.zxs * parts["I"]) + TWO_PI * np.abs(f.ps)
          + np.abs(parts["src"]))
    px = 1.0 + f.pxs
    s1 = (0.5 * ((1 + f.zxs ** 2) * f.pys ** 2 + (1 + f.zys ** 2) * px ** 2
                 + 2 * np.abs(f.zxs * f.zys * px * f.pys)) / (1 + f.zxs ** 2 + f.zys ** 2)
          + np.abs(f.zs) / prob.F ** 2 + 0.5)
    x1, dx, nu = prob.x1, prob.dx, prob.nu
    psix, zetax = f.psix, f.zetax
    s4 = np.abs(x1 / dx) * (np.abs(psix[:, 1]) + np.abs(psix[:, 0])) + nu * np.abs(psix[:, 0])
    s6 = np.abs(x1 / dx) * (np.abs(zetax[:, 1]) + np.abs(zetax[:, 0])) + nu * np.abs(zetax[:, 0])
    return np.fmax(1.0, pack(s1, s2, s4, s6))


def residual_full_domain(prob: Problem, psix_full, zetax_full):
    """Residual on the whole strip y in [-y_M, y_M] (2M-1 rows), with no image
    terms and not-a-knot spline ends: the boundary-integral equation taken
    over the full (x, y) plane, truncated.  Used to check the image terms of
    the half-domain form.  Returns (E1, E2, E4, E6) as (2M-1)-row arrays."""
    return _residual_geom(prob, _full_geom(prob), psix_full, zetax_full)


def even_extension(a):
    """Rows l = 1..M of a half-domain array -> rows for y = -y_M..y_M."""
    return np.concatenate([a[:0:-1], a], axis=0)


def zeta_grid(prob: Problem, u):
    """Free-surface heights zeta_{k,l} on the mesh for a reduced state u."""
    psix, zetax = unpack(prob, u)
    return trapezoid_rows(zetax, (-prob.x1 / prob.nu) * zetax[:, 0], prob.dx)
