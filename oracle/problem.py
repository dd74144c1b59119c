"""Problem definition for the CPU oracle: mesh, truncated domain, parameters.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package;
only tests/, the smoke check and the benchmark's CPU-baseline leg use it.

Numerical discretisation section: an N x M regular mesh (x_k, y_l) with
spacings dx, dy on the truncated rectangle x_1 <= x <= x_N, y_1 <= y <= y_M.
Half-mesh collocation points are (x_{k+1/2}, y_l), k = 1..N-1, l = 1..M.
The half domain y >= 0 is used with image terms, so y_1 = 0.

Upstream decay constant nu (the paper's n in the radiation condition) is 0.05.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class Problem:
    N: int
    M: int
    x1: float
    xN: float
    yM: float
    F: float
    eps: float
    nu: float = 0.05
    weights: str = "trapezoid"          # "trapezoid" | "simpson"
    spline_bc: str = "clamped0"         # "clamped0" (s=0 at y=0, not-a-knot at y_M) | "notaknot"

    def __post_init__(self):
        if self.N < 4 or self.M < 4:
            raise ValueError("N and M must be >= 4")
        if self.weights not in ("trapezoid", "simpson"):
            raise ValueError("weights must be 'trapezoid' or 'simpson'")
        if self.weights == "simpson" and (self.N % 2 == 0 or self.M % 2 == 0):
            raise ValueError("Simpson weights need odd N and M")
        if self.spline_bc not in ("clamped0", "notaknot"):
            raise ValueError("spline_bc must be 'clamped0' or 'notaknot'")
        if not (self.x1 < self.xN) or self.yM <= 0 or self.F <= 0 or self.eps < 0:
            raise ValueError("bad domain or parameters")

    # --- mesh -----------------------------------------------------------
    @property
    def dx(self) -> float:
        return (self.xN - self.x1) / (self.N - 1)

    @property
    def dy(self) -> float:
        return self.yM / (self.M - 1)

    @property
    def n_unknowns(self) -> int:
        return 2 * self.N * self.M

    def x(self) -> np.ndarray:
        """Grid abscissae x_k = x_1 + (k-1) dx."""
        return self.x1 + np.arange(self.N) * self.dx

    def y(self) -> np.ndarray:
        """Grid ordinates y_l = (l-1) dy."""
        return np.arange(self.M) * self.dy

    def xs(self) -> np.ndarray:
        """Collocation abscissae x*_k = x_{k+1/2} = x_1 + (k - 1/2) dx."""
        return self.x1 + (np.arange(self.N - 1) + 0.5) * self.dx

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def rule_weights(n: int, h: float, rule: str) -> np.ndarray:
    """One-dimensional composite quadrature weights on n equally spaced points.

    Trapezoid: h * (1/2, 1, ..., 1, 1/2).  Simpson: h/3 * (1, 4, 2, ..., 2, 4, 1).
    The two-dimensional weight w(i,j) is the product of the x and y rules
    (numerical discretisation section, where the integrals are discretised
    with the trapezoidal rule; Simpson is the alternative weighting scheme).
    """
    if rule == "trapezoid":
        c = np.ones(n)
        c[0] = c[-1] = 0.5
        return h * c
    if rule == "simpson":
        if n % 2 == 0:
            raise ValueError("Simpson rule needs an odd number of points")
        c = np.ones(n)
        c[1:-1:2] = 4.0
        c[2:-1:2] = 2.0
        return h * c / 3.0
    raise ValueError(rule)


def weights(prob: Problem) -> np.ndarray:
    """w(i,j) as an (M, N) array (row l, column k)."""
    wx = rule_weights(prob.N, prob.dx, prob.weights)
    wy = rule_weights(prob.M, prob.dy, prob.weights)
    return wy[:, None] * wx[None, :]


def flat_state(prob: Problem) -> np.ndarray:
    """Flat-surface initial guess (Jacobian-free Newton-Krylov overview):
    phi_x = 1, zeta_x = 0 at every mesh point.  In the reduced unknown vector
    (phi_{1,l} and zeta_{1,l} eliminated by the first and third radiation
    equations) this is [1,...,1, 0,...,0]."""
    NM = prob.N * prob.M
    u = np.zeros(2 * NM)
    u[:NM] = 1.0
    return u
