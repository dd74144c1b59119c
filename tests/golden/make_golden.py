"""Writes the stored inputs under tests/golden/ by calling only the oracle.

config2_linear_state.npy: the root of the discrete linear system (the
linearised problem of the paper's linear-problem section, discretised as in
Appendix B) on the 181 x 61 mesh, x in [-16, 8], y in [0, 12], eps = 0.1,
F = 0.7, i.e. u_flat - eps J_lin^{-1} s, solved through the Schur complement
of Appendix C with all of D kept.  It seeds the residual-throughput batch
(linear solution plus N(0, 1e-3^2) noise).

Run:  python tests/golden/make_golden.py
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Problem  # noqa: E402
from oracle.linear import linear_solution  # noqa: E402


def main():
    t = time.time()
    prob = Problem(181, 61, -16.0, 8.0, 12.0, F=0.7, eps=0.1)
    u = linear_solution(prob)
    path = os.path.join(HERE, "config2_linear_state.npy")
    np.save(path, u, allow_pickle=False)
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    with open(path + ".sha256", "w") as f:
        f.write(f"{digest}  config2_linear_state.npy\n")
    print(f"wrote {path} ({u.size} values) in {time.time() - t:.1f} s, sha256 {digest}")


if __name__ == "__main__":
    main()
