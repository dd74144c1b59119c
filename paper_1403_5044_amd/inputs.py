"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Plain data only: mesh/domain/physics settings of the workloads,
the flat initial state and seeded perturbations.  No arithmetic of the method
lives here.

Workloads (meshes and domains; the paper's results section and Table 1 give
the shapes this suite is modelled on):
  W31X11    31 x 11   x in [-8, 8],   y in [0, 8],   eps 0.05, F 0.7
  W181X61   181 x 61  x in [-16, 8],  y in [0, 12],  eps 0.1,  F 0.7
  W361X121  361 x 121 x in [-14, 40], y in [0, 18],  F in {0.5, 0.7, 1.0}, eps in {0.1, 0.3}
  W721X241  721 x 241 x in [-14, 40], y in [0, 18],  F 0.7, eps 0.1 .. 0.5
  W721X241_F14  721 x 241 x in [-56, 160], y in [0, 72], F 1.4, eps 1 (spacing 0.3)
  serving   meshes {61x21, 121x41, 181x61, 241x81} on x in [-16, 8], y in [0, 12],
           F ~ U[0.5, 1.0], eps ~ U[0.05, 0.4], Poisson arrivals
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")

W31X11 = dict(N=31, M=11, x1=-8.0, xN=8.0, yM=8.0, F=0.7, eps=0.05)
W181X61 = dict(N=181, M=61, x1=-16.0, xN=8.0, yM=12.0, F=0.7, eps=0.1)
W361X121 = dict(N=361, M=121, x1=-14.0, xN=40.0, yM=18.0, F=0.7, eps=0.1)
W361X121_F = (0.5, 0.7, 1.0)
W361X121_EPS = (0.1, 0.3)
W721X241 = dict(N=721, M=241, x1=-14.0, xN=40.0, yM=18.0, F=0.7, eps=0.1)
W721X241_EPS = (0.1, 0.2, 0.3, 0.4, 0.5)
# F = 1.4 on 721 x 241 with spacing 0.3 from x_1 = -56 (the paper's F = 1.4 surface)
W721X241_F14 = dict(N=721, M=241, x1=-56.0, xN=160.0, yM=72.0, F=1.4, eps=1.0)
# Block half-bandwidth of the preconditioner on the paper's domain: the band that
# matters is a distance in y (1.2 here), so it doubles when the spacing halves
Q_BLOCKS = {(361, 121): 8, (721, 241): 16}
# Solver settings of the large-mesh solves (361 x 121 and beyond)
LARGE_SOLVE = dict(tol=1e-10, max_gmres=600, gmres_restart=60, max_newton=20)
SERVING_MESHES = ((61, 21), (121, 41), (181, 61), (241, 81))
SERVING_DOMAIN = dict(x1=-16.0, xN=8.0, yM=12.0)
# Table 1 meshes (every row at eps = 1, F = 0.7); spacing 0.3 (91 x 31, x_1 = -9)
# and 0.15 (361 x 121, x_1 = -14) are printed, the others are filled in at the
# spacing of the nearest printed mesh.
TABLE1 = {(91, 31): dict(x1=-9.0, xN=18.0, yM=9.0), (181, 61): dict(x1=-16.0, xN=8.0, yM=12.0),
          (271, 91): dict(x1=-13.5, xN=27.0, yM=13.5), (361, 121): dict(x1=-14.0, xN=40.0, yM=18.0),
          (451, 151): dict(x1=-14.0, xN=53.5, yM=22.5)}


def flat_state(N: int, M: int) -> np.ndarray:
    """phi_x = 1, zeta_x = 0 (the flat-surface initial guess)."""
    u = np.zeros(2 * N * M)
    u[:N * M] = 1.0
    return u


def perturbed(base: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """base + N(0, sigma^2) i.i.d. on every entry, numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return base + sigma * rng.standard_normal(base.size)


def smooth_state(N: int, M: int, amp: float, seed: int) -> np.ndarray:
    """A flat state plus a seeded smooth perturbation of phi_x and zeta_x
    (random low-order Fourier modes), for parity checks away from the flat state."""
    rng = np.random.default_rng(seed)
    x = np.linspace(0.0, 1.0, N)[None, :]
    y = np.linspace(0.0, 1.0, M)[:, None]
    u = flat_state(N, M)
    for part in range(2):
        f = np.zeros((M, N))
        for _ in range(4):
            kx, ky = rng.integers(1, 5, 2)
            a, ph = rng.normal(), rng.uniform(0, 2 * np.pi)
            f += a * np.sin(np.pi * kx * x + ph) * np.cos(np.pi * ky * y)
        u[part * N * M:(part + 1) * N * M] += amp * f.ravel()
    return u


def linear_state_181x61() -> np.ndarray:
    """The discrete linear solution of the 181 x 61 workload (eps = 0.1), written by
    tests/golden/make_golden.py; its SHA-256 is checked on load."""
    path = os.path.join(GOLDEN, "linear_state_181x61.npy")
    with open(path + ".sha256") as f:
        want = f.read().split()[0]
    raw = open(path, "rb").read()
    if hashlib.sha256(raw).hexdigest() != want:
        raise RuntimeError("linear_state_181x61.npy does not match its hash")
    return np.load(path, allow_pickle=False)


def batch_181x61(n: int = 16) -> list[np.ndarray]:
    """The residual-throughput batch: linear solution + N(0, 1e-3 ** 2), seeds 0..n-1."""
    base = linear_state_181x61()
    return [perturbed(base, 1e-3, s) for s in range(n)]


def serving_requests(n: int = 256, rate_hz: float = 20.0, seed: int = 0):
    """n requests with Poisson arrivals at rate_hz: (t_arrival, N, M, F, eps)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    mesh = rng.integers(0, len(SERVING_MESHES), n)
    F = rng.uniform(0.5, 1.0, n)
    eps = rng.uniform(0.05, 0.4, n)
    return [(float(t[i]), *SERVING_MESHES[mesh[i]], float(F[i]), float(eps[i])) for i in range(n)]
