"""Root finding for E(u) = 0 in the oracle: damped Newton, GMRES, JFNK.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

The method (Jacobian-free Newton-Krylov section) is a fast route to the root
of the discrete system E(u) = 0 (eq. nonlinearsys).  Up to the solver
tolerance the root does not depend on GMRES, the preconditioner, the shift h
or the line search, so the oracle may use exact directional derivatives
(complex step) and tight inner tolerances.

  * damped Newton: u_{k+1} = u_k + lambda_k du_k (eq. newtonstep0) with
    lambda_k in (0, 1] halved until ||E|| decreases sufficiently;
  * the Newton step solves J du = -E (eq. newtonstep), either densely
    (Jacobian from complex-step columns, tiny meshes) or with right-
    preconditioned GMRES (Krylov space K_m(J P^{-1}, E));
  * epsilon continuation: each root is the initial guess for the next eps.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .problem import Problem, flat_state
from .equations import residual
from .linear import BlockPreconditioner

CS_STEP = 1e-30


def jvp_complex(prob: Problem, u, z):
    """Exact directional derivative J(u) z = Im E(u + i h z) / h."""
    nz = np.linalg.norm(z)
    if nz == 0.0:
        return np.zeros_like(u)
    zz = z / nz
    return residual(prob, u + 1j * CS_STEP * zz).imag / CS_STEP * nz


def jvp_fd(prob: Problem, u, Eu, z, h):
    """First-order difference quotient (eq. JvApprox): (E(u + h z) - E(u)) / h."""
    return (residual(prob, u + h * z) - Eu) / h


def jacobian_complex(prob: Problem, u):
    n = u.size
    J = np.empty((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        J[:, i] = residual(prob, u + 1j * CS_STEP * e).imag / CS_STEP
        e[i] = 0.0
    return J


def gmres(matvec, b, psolve, *, tol: float, restart: int = 30, maxiter: int = 600):
    """Right-preconditioned restarted GMRES (Saad & Schultz), modified Gram-Schmidt
    Arnoldi with Givens rotations.  Solves A x = b with A P^{-1} y = b, x = P^{-1} y.
    Stops when ||b - A x||_2 <= tol.  Returns (x, iterations, final residual norm)."""
    n = b.size
    x = np.zeros(n)
    r = b.copy()
    beta = np.linalg.norm(r)
    its = 0
    while its < maxiter:
        if beta <= tol:
            break
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            w = matvec(psolve(V[j]))
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            if abs(g[j + 1]) <= tol or its >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + psolve(V[:j_done].T @ y)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    return x, its, beta


@dataclass
class SolveInfo:
    converged: bool = False
    newton: int = 0
    gmres: int = 0
    evals: int = 0
    norms: list = field(default_factory=list)


def newton(prob: Problem, u0, *, tol: float = 1e-10, max_newton: int = 50,
           linear: str = "gmres", q: int | None = None, pre: BlockPreconditioner | None = None,
           eta: float = 1e-8, alpha: float = 1e-4, lam_min: float = 1e-4):
    """Damped Newton iteration to ||E||_inf <= tol.

    linear = "dense": exact Jacobian (complex-step columns) and a dense solve;
    linear = "gmres": JFNK with exact JVPs and the linear-Jacobian block
    preconditioner with block half-bandwidth q (default: dense, q = M-1).
    Line search: lambda halves until ||E(u + lambda du)||_2 <= (1 - alpha lambda) ||E(u)||_2."""
    u = np.array(u0, dtype=float, copy=True)
    info = SolveInfo()
    E = residual(prob, u)
    info.evals += 1
    if linear == "gmres" and pre is None:
        pre = BlockPreconditioner(prob, prob.M - 1 if q is None else q)
    while True:
        enorm = np.abs(E).max()
        info.norms.append(enorm)
        if enorm <= tol:
            info.converged = True
            return u, info
        if info.newton >= max_newton:
            return u, info
        if linear == "dense":
            du = np.linalg.solve(jacobian_complex(prob, u), -E)
            info.evals += u.size
        else:
            uu = u

            def mv(v):
                return jvp_complex(prob, uu, v)

            b = -E
            du, its, _ = gmres(mv, b, pre.solve, tol=eta * np.linalg.norm(b))
            info.gmres += its
            info.evals += its + 1
        n0 = np.linalg.norm(E)
        lam = 1.0
        while True:
            un = u + lam * du
            En = residual(prob, un)
            info.evals += 1
            if np.all(np.isfinite(En)) and np.linalg.norm(En) <= (1.0 - alpha * lam) * n0:
                break
            lam *= 0.5
            if lam < lam_min:
                return u, info
        u, E = un, En
        info.newton += 1


def continuation(prob: Problem, eps_list, u0=None, **kw):
    """Bootstrap in eps: the root at each eps is the initial guess for the next."""
    u = flat_state(prob) if u0 is None else np.array(u0, dtype=float)
    out = []
    for e in eps_list:
        p = prob.with_(eps=float(e))
        u, info = newton(p, u, **kw)
        out.append((e, u.copy(), info))
        if not info.converged:
            break
    return out
