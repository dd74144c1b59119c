"""Writes the stored inputs and expected values under tests/golden/ by calling
only the oracle.

linear_state_181x61.npy: the root of the discrete linear system (the
linearised problem of the paper's linear-problem section, discretised as in
Appendix B) on the 181 x 61 mesh, x in [-16, 8], y in [0, 12], eps = 0.1,
F = 0.7, i.e. u_flat - eps J_lin^{-1} s, solved through the Schur complement
of Appendix C with all of D kept.  It seeds the residual-throughput batch
(linear solution plus N(0, 1e-3^2) noise).

root_181x61.npy: the root of the nonlinear system E(u) = 0 on the same mesh
and parameters, by the oracle's damped Newton (exact complex-step JVPs, GMRES
preconditioned by the full linear Jacobian) to ||E||_inf <= 1e-12, started
from the linear solution (the eps-continuation path from the flat surface:
the linear solution is the first-order term of that path).  The converged
surface heights zeta are compared with the GPU solve.

table1_91x31_eps1_root.npy: the root at eps = 1, F = 0.7 on the 91 x 31 mesh of
the paper's results section (spacing 0.3, x_1 = -9, so x in [-9, 18] and
y in [0, 9]), reached by eps continuation in steps of 0.1 from the flat
surface (each root starts the next Newton solve; the bootstrapping paragraph
of the JFNK overview), every step to ||E||_inf <= 1e-12 with the full linear
Jacobian as preconditioner.

Each file is stored with its SHA-256.

Run:  python tests/golden/make_golden.py [linear] [root] [table1]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Problem  # noqa: E402
from oracle.linear import BlockPreconditioner, linear_solution  # noqa: E402
from oracle.solve import continuation, newton  # noqa: E402


def _store(name, arr):
    path = os.path.join(HERE, name)
    np.save(path, arr, allow_pickle=False)
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    with open(path + ".sha256", "w") as f:
        f.write(f"{digest}  {name}\n")
    return path, digest


def problem_181x61():
    return Problem(181, 61, -16.0, 8.0, 12.0, F=0.7, eps=0.1)


def make_linear():
    t = time.time()
    u = linear_solution(problem_181x61())
    path, digest = _store("linear_state_181x61.npy", u)
    print(f"wrote {path} ({u.size} values) in {time.time() - t:.1f} s, sha256 {digest}")


def make_root():
    t = time.time()
    prob = problem_181x61()
    pre = BlockPreconditioner(prob, prob.M - 1)
    u0 = linear_solution(prob, pre)
    u, info = newton(prob, u0, tol=1e-12, pre=pre, eta=1e-6)
    if not info.converged:
        raise RuntimeError(f"oracle Newton did not converge: {info}")
    path, digest = _store("root_181x61.npy", u)
    print(f"wrote {path} in {time.time() - t:.1f} s: {info.newton} Newton, {info.gmres} GMRES, "
          f"norms {['%.2e' % v for v in info.norms]}, sha256 {digest}")


def make_table1_root():
    t = time.time()
    prob = Problem(91, 31, -9.0, 18.0, 9.0, F=0.7, eps=1.0)
    pre = BlockPreconditioner(prob, prob.M - 1)
    steps = continuation(prob, [0.1 * k for k in range(1, 11)], tol=1e-12, pre=pre, eta=1e-6)
    for e, _, info in steps:
        print(f"  eps {e:.1f}: converged {info.converged}, {info.newton} Newton, "
              f"{info.gmres} GMRES, final {info.norms[-1]:.2e}", flush=True)
    e, u, info = steps[-1]
    if not info.converged or abs(e - 1.0) > 1e-12:
        raise RuntimeError(f"oracle continuation stopped at eps {e}: {info}")
    path, digest = _store("table1_91x31_eps1_root.npy", u)
    print(f"wrote {path} in {time.time() - t:.1f} s, sha256 {digest}")


if __name__ == "__main__":
    which = sys.argv[1:] or ["linear", "root", "table1"]
    if "linear" in which:
        make_linear()
    if "root" in which:
        make_root()
    if "table1" in which:
        make_table1_root()
