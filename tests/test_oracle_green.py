"""Pin of the double-layer term of the oracle's all-pairs sum by Green's second
identity.  CPU only.

The boundary-integral equation (eq. IntegroEqn) is Green's second identity for
the perturbation potential on the free surface z = zeta(x, y), with the fluid
below it.  For ANY function u harmonic in the fluid and decaying at infinity,
and P = (x*, y*, zeta*) on the surface, the identity reads

    2 pi u(P) = int (1/R) du/dn dS + int u K1 dx dy,

where du/dn dS = (-u_x zeta_x - u_y zeta_y + u_z) dx dy (normal (-zeta_x,
-zeta_y, 1), out of the fluid) and K1 is the direct part of the paper's kernel.
Splitting u K1 = (u - u*) K1 + u* K1 isolates the oracle's double-layer term
Sum_ij w_ij (u_ij - u*) K1_ij, which vanishes at the flat state and is O(eps^2)
at the root, so no other pin reaches it.

Here u = 1/|X - X0| with X0 above a smooth Gaussian bump, on the full strip
with no images.  The single layer, the solid-angle integral int K1 and the flat
exterior beyond the truncated rectangle are integrated independently by
adaptive polar quadrature about (x*, y*) (the integrands times the polar
Jacobian are bounded); the double layer comes from the oracle's pair_sum as the
difference of two sums that share every other term.  The identity then fixes
the double layer's sign, weight and the subtracted u*.
"""
import inspect
import textwrap

import numpy as np
import pytest
from scipy import integrate

from oracle import equations as R

A_BUMP, S_BUMP = 0.3, 1.5          # zeta = a exp(-(x^2 + y^2) / s^2)
X0 = np.array([0.3, 0.0, 1.0])    # pole of u, above the bump (max zeta = 0.3)
HALF = 12.0                        # truncated rectangle [-12, 12]^2
XS, YS = 0.45, 0.3                 # collocation point: on the bump's flank


def _zeta(x, y):
    return A_BUMP * np.exp(-(x * x + y * y) / S_BUMP ** 2)


def _slopes(x, y):
    z = _zeta(x, y)
    return -2.0 * x / S_BUMP ** 2 * z, -2.0 * y / S_BUMP ** 2 * z


def _u_grad(x, y, z):
    d = np.stack([x - X0[0], y - X0[1], z - X0[2]])
    r = np.sqrt((d * d).sum(axis=0))
    return 1.0 / r, -d / r ** 3


def _edge(t, xs, ys):
    """Distance from (xs, ys) to the rectangle's boundary along angle t."""
    c, s = np.cos(t), np.sin(t)
    cand = []
    if c > 0:
        cand.append((HALF - xs) / c)
    if c < 0:
        cand.append((-HALF - xs) / c)
    if s > 0:
        cand.append((HALF - ys) / s)
    if s < 0:
        cand.append((-HALF - ys) / s)
    return min(cand)


def _corner_breaks(xs, ys):
    br = sorted(np.arctan2(cy - ys, cx - xs) % (2 * np.pi)
                for cx in (-HALF, HALF) for cy in (-HALF, HALF))
    return list(zip(br, br[1:] + [br[0] + 2 * np.pi]))


def _polar_inside(f, xs, ys):
    """Integral of f(x, y) over the rectangle, polar about (xs, ys)."""
    def radial(t):
        re = _edge(t, xs, ys)
        c, s = np.cos(t), np.sin(t)
        pts = [p for p in (0.5, 1.0, 2.0, 4.0) if p < re]
        return integrate.quad(lambda r: f(xs + r * c, ys + r * s) * r, 0.0, re, epsabs=0,
                              epsrel=1e-11, limit=400, points=pts)[0]
    return sum(integrate.quad(radial, t0, t1, epsabs=0, epsrel=1e-11, limit=400)[0]
               for t0, t1 in _corner_breaks(xs, ys))


def _polar_outside(f, xs, ys):
    """Integral of f over the plane outside the rectangle, r = edge / t, t in (0, 1]."""
    def radial(t):
        re = _edge(t, xs, ys)
        c, s = np.cos(t), np.sin(t)

        def g(tt):
            r = re / tt
            return f(xs + r * c, ys + r * s) * r * re / (tt * tt)
        return integrate.quad(g, 0.0, 1.0, epsabs=0, epsrel=1e-11, limit=400)[0]
    return sum(integrate.quad(radial, t0, t1, epsabs=0, epsrel=1e-11, limit=400)[0]
               for t0, t1 in _corner_breaks(xs, ys))


def _continuous_terms():
    """u*, int K1 (rectangle), single layer (rectangle), exterior (flat: zeta = 0)."""
    zs = _zeta(XS, YS)
    us = float(_u_grad(np.array(XS), np.array(YS), np.array(zs))[0])

    def k1(x, y):
        zx, zy = _slopes(x, y)
        dx, dy, dz = x - XS, y - YS, _zeta(x, y) - zs
        return (dz - dx * zx - dy * zy) / (dx * dx + dy * dy + dz * dz) ** 1.5

    def single(x, y):
        z = _zeta(x, y)
        zx, zy = _slopes(x, y)
        _, g = _u_grad(x, y, z)
        return (-g[0] * zx - g[1] * zy + g[2]) / np.sqrt((x - XS) ** 2 + (y - YS) ** 2
                                                          + (z - zs) ** 2)

    def exterior(x, y):
        u, g = _u_grad(x, y, 0.0 * x)
        r = np.sqrt((x - XS) ** 2 + (y - YS) ** 2 + zs * zs)
        return g[2] / r + u * (-zs) / r ** 3

    def double(x, y):
        u, _ = _u_grad(x, y, _zeta(x, y))
        return (u - us) * k1(x, y)

    return dict(us=us, omega=_polar_inside(k1, XS, YS), single=_polar_inside(single, XS, YS),
                exterior=_polar_outside(exterior, XS, YS), double=_polar_inside(double, XS, YS))


@pytest.fixture(scope="module")
def cont():
    return _continuous_terms()


def _discrete_double_layer(h, images, pair_sum=None):
    """Sum_ij w (u_ij - u*) K1_ij at (XS, YS) from the oracle's pair_sum, as the
    difference of two sums that differ only in u (the K2 and S2 terms cancel)."""
    pair_sum = pair_sum or R.pair_sum
    n = int(round(2 * HALF / h)) + 1
    x = -HALF + np.arange(n) * h
    k = int(round((XS + HALF) / h - 0.5))
    assert abs(-HALF + (k + 0.5) * h - XS) < 1e-12
    wx = np.full(n, h)
    wx[0] = wx[-1] = h / 2
    if images:      # rows y >= 0 with mirror terms; the row y = 0 carries weight h/2
        R_ = (n + 1) // 2
        yidx = np.arange(R_)
    else:           # the whole strip
        R_ = n
        yidx = np.arange(n) - (n - 1) // 2
    wy = np.full(R_, h)
    wy[0] = wy[-1] = h / 2
    geom = R._Geom(n, R_, -HALF, HALF, h, h, yidx, wx, wy, -HALF, HALF, images, "notaknot")
    l = int(np.flatnonzero(np.abs(geom.y - YS) < 1e-12)[0])
    X, Y = np.meshgrid(x, geom.y)
    Z = _zeta(X, Y)
    ZX, ZY = _slopes(X, Y)
    U = _u_grad(X, Y, Z)[0]
    zs = _zeta(XS, YS)
    zxs, zys = _slopes(XS, YS)

    def at_point(v):
        a = np.full((R_, n - 1), np.nan)
        a[l, k] = v
        return a

    us = float(_u_grad(np.array(XS), np.array(YS), np.array(zs))[0])
    common = dict(psix=None, zetax=ZX, zeta=Z, psiy=None, zetay=ZY, pxs=None, pys=None,
                  zs=at_point(zs), zxs=at_point(zxs), zys=at_point(zys))
    f = R.Fields(psi=U, ps=at_point(us), **common)
    f0 = R.Fields(psi=0.0 * U, ps=at_point(0.0), **common)
    c = l * (n - 1) + k
    return pair_sum(geom, f, cols=[c])[l, k] - pair_sum(geom, f0, cols=[c])[l, k]


def test_continuous_greens_identity_holds_for_the_quadratures(cont):
    """The independent quadratures satisfy 2 pi u* = DL + u* Omega + SL + exterior,
    which confirms the kernel sign and the identity used below."""
    lhs = cont["double"] + cont["us"] * cont["omega"] + cont["single"] + cont["exterior"]
    assert abs(lhs - 2 * np.pi * cont["us"]) <= 1e-9


def _green_error(D, cont):
    return D + cont["us"] * cont["omega"] + cont["single"] + cont["exterior"] \
        - 2 * np.pi * cont["us"]


def test_double_layer_of_the_pair_sum_satisfies_greens_identity(cont):
    """Refining h = 0.3, 0.1, 1/30 (collocation point fixed at a half-mesh
    point) drives the oracle's double layer to the value Green's identity
    requires; observed errors 6.5e-5, 3.5e-6, 2.8e-7 (at least a factor 9 per
    refinement by 3)."""
    errs = [abs(_green_error(_discrete_double_layer(h, False), cont))
            for h in (0.3, 0.1, 1.0 / 30)]
    assert errs[0] > 5 * errs[1] and errs[1] > 5 * errs[2]
    assert errs[2] <= 1e-6
    # the term is not small: a sign or weight error could not hide in the tolerance
    assert abs(cont["double"]) > 0.3


def test_double_layer_with_images_equals_the_full_strip():
    """The half domain with mirror terms gives the same double layer for a surface
    and potential that are even in y."""
    for h in (0.3, 0.1):
        full = _discrete_double_layer(h, False)
        half = _discrete_double_layer(h, True)
        assert abs(full - half) <= 1e-13 * max(1.0, abs(full))


_T1 = "t1 = w[None, :] * (psi[None, :] - ps[sl, None]) * K1"
MUTANTS = {
    "flipped sign": "t1 = -w[None, :] * (psi[None, :] - ps[sl, None]) * K1",
    "dropped weight": "t1 = (psi[None, :] - ps[sl, None]) * K1",
    "psi* not subtracted": "t1 = w[None, :] * psi[None, :] * K1",
    "collocation slopes in K1": None,   # built below
}


def _mutant_pair_sum(name):
    src = textwrap.dedent(inspect.getsource(R.pair_sum))
    if name == "collocation slopes in K1":
        old = "zx[None, :], zy[None, :],"
        assert old in src
        src = src.replace(old, "zxs[sl, None], zys[sl, None],")
    else:
        assert _T1 in src
        src = src.replace(_T1, MUTANTS[name])
    scope = dict(vars(R))
    exec(compile(src, "<mutant pair_sum>", "exec"), scope)
    return scope["pair_sum"]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_in_the_double_layer_fail_the_pin(cont, name):
    """Each mistake, planted in a scratch copy of pair_sum, moves the error at
    h = 0.1 far above the pin's tolerance."""
    D = _discrete_double_layer(0.1, False, pair_sum=_mutant_pair_sum(name))
    assert abs(_green_error(D, cont)) > 1e-3
