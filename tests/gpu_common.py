"""Helpers for the GPU tests: converting problems between the product binding
and the oracle, and moving arrays.  The two sides share only the seeded
input generators (paper_1403_5044_amd.inputs)."""
import numpy as np
import torch

from oracle import Problem as OProblem
from paper_1403_5044_amd import api


def oprob(p: api.Problem) -> OProblem:
    return OProblem(p.N, p.M, p.x1, p.xN, p.yM, F=p.F, eps=p.eps, nu=p.nu, weights=p.weights,
                    spline_bc=p.spline_bc)


def gprob(cfg: dict, **kw) -> api.Problem:
    d = dict(cfg)
    d.update(kw)
    return api.Problem(**d)


def dev(x: np.ndarray) -> torch.Tensor:
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_residual(p: api.Problem, u: np.ndarray) -> np.ndarray:
    return host(api.residual(p, dev(u)))


def log(msg: str):
    print(msg, flush=True)
