"""Thin Python binding over libshipwave: argument marshalling only.

Tensors are torch tensors on the GPU (float64, contiguous); the library works
on their device pointers on the current torch stream.  Every numerical step
runs in the HIP library; if it is not built, the calls raise.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, replace

import torch

from . import _lib as L

WEIGHTS = {"trapezoid": 0, "simpson": 1}
SPLINE = {"clamped0": 0, "notaknot": 1}
PRECISION = {"fp64": 0, "fp32": 1}


@dataclass(frozen=True)
class Problem:
    """Mesh N x M on [x1, xN] x [0, yM]; Froude number F, source strength eps."""
    N: int
    M: int
    x1: float
    xN: float
    yM: float
    F: float
    eps: float
    nu: float = 0.05
    weights: str = "trapezoid"
    spline_bc: str = "clamped0"
    precision: str = "fp64"

    @property
    def n_unknowns(self) -> int:
        return 2 * self.N * self.M

    @property
    def pairs(self) -> int:
        """(collocation, grid) pairs in one all-pairs sum."""
        return (self.N - 1) * self.M * self.N * self.M

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)

    def c_struct(self) -> L.SwProblem:
        p = L.SwProblem()
        p.mesh.N, p.mesh.M = self.N, self.M
        p.domain.x1, p.domain.xN, p.domain.yM = self.x1, self.xN, self.yM
        p.params.F, p.params.eps, p.params.nu = self.F, self.eps, self.nu
        p.params.weights = WEIGHTS[self.weights]
        p.params.spline_bc = SPLINE[self.spline_bc]
        p.params.precision = PRECISION[self.precision]
        p.params.reserved = 0
        return p


def _lib():
    return L.load()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, n: int, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous float64 with {n} elements")
    return t.data_ptr()


def residual(prob: Problem, u: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """E(u) (reduced Appendix-A order)."""
    lib = _lib()
    n = prob.n_unknowns
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=u.device)
    ps = prob.c_struct()
    L.check(lib.shipwave_residual(C.byref(ps), _dev(u, n, "u"), _dev(out, n, "E"), _stream()))
    return out


def residual_noalloc(prob: Problem, u: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """E(u) through the entry point that allocates nothing (the library's fixed array)."""
    lib = _lib()
    n = prob.n_unknowns
    ps = prob.c_struct()
    L.check(lib.shipwave_residual_noalloc(C.byref(ps), _dev(u, n, "u"), _dev(out, n, "E"),
                                          _stream()))
    return out


def residual_batched(probs, us, outs=None):
    """E(u_b) for several problems in shared launches."""
    lib = _lib()
    nb = len(probs)
    if outs is None:
        outs = [torch.empty(p.n_unknowns, dtype=torch.float64, device=u.device)
                for p, u in zip(probs, us)]
    arr = (L.SwProblem * nb)(*[p.c_struct() for p in probs])
    up = (C.c_void_p * nb)(*[_dev(u, p.n_unknowns, "u") for p, u in zip(probs, us)])
    ep = (C.c_void_p * nb)(*[_dev(e, p.n_unknowns, "E") for p, e in zip(probs, outs)])
    L.check(lib.shipwave_residual_batched(nb, arr, up, ep, _stream()))
    return outs


def jvp(prob: Problem, u, Eu, z, h: float = 0.0, out=None):
    """(E(u + h z) - Eu) / h; h <= 0 picks the step from the norms of u and z."""
    lib = _lib()
    n = prob.n_unknowns
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=u.device)
    ps = prob.c_struct()
    L.check(lib.shipwave_jvp(C.byref(ps), _dev(u, n, "u"), _dev(Eu, n, "Eu"), _dev(z, n, "z"),
                             float(h), _dev(out, n, "Jz"), _stream()))
    return out


def zeta(prob: Problem, u, out=None):
    lib = _lib()
    n = prob.n_unknowns
    if out is None:
        out = torch.empty(prob.N * prob.M, dtype=torch.float64, device=u.device)
    ps = prob.c_struct()
    L.check(lib.shipwave_zeta(C.byref(ps), _dev(u, n, "u"),
                              _dev(out, prob.N * prob.M, "zeta"), _stream()))
    return out


def profile_enable(on: bool = True):
    """Start (clear) or stop event timing of the all-pairs kernel launches."""
    L.check(_lib().shipwave_profile_enable(1 if on else 0))


def profile_read():
    """(launches, total kernel milliseconds, total pairs) since profile_enable(True)."""
    n = C.c_int64()
    ms = C.c_double()
    pr = C.c_double()
    L.check(_lib().shipwave_profile_read(C.byref(n), C.byref(ms), C.byref(pr)))
    return n.value, ms.value, pr.value


def debug_inject_nonfinite(kinds: int, nth: int):
    """Host-forced NaN in the nth evaluation of each kind in `kinds` (bit 1 initial
    residual, 2 line-search trial, 4 FP64 JVP point, 8 FP32 JVP point) of every later
    solve; (0, 0) switches it off.  For tests of the failure paths."""
    L.check(_lib().shipwave_debug_inject_nonfinite(int(kinds), int(nth)))


class Preconditioner:
    """Linear-Jacobian block preconditioner with block half-bandwidth q."""

    def __init__(self, prob: Problem, q: int):
        self.lib = _lib()
        self.prob = prob
        self.q = q
        h = C.c_void_p()
        ps = prob.c_struct()
        L.check(self.lib.shipwave_precond_build_banded(C.byref(ps), int(q), C.byref(h), _stream()))
        self.handle = h

    def apply(self, b, out=None):
        n = self.prob.n_unknowns
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=b.device)
        L.check(self.lib.shipwave_precond_apply(self.handle, _dev(b, n, "b"), _dev(out, n, "x"),
                                                _stream()))
        return out

    @staticmethod
    def apply_batched(pcs, bs, outs=None):
        """x_i = P_i^{-1} b_i for several preconditioners in shared launches."""
        n = len(pcs)
        if outs is None:
            outs = [torch.empty(p.prob.n_unknowns, dtype=torch.float64, device=b.device)
                    for p, b in zip(pcs, bs)]
        hp = (C.c_void_p * n)(*[p.handle.value for p in pcs])
        bp = (C.c_void_p * n)(*[_dev(b, p.prob.n_unknowns, "b") for p, b in zip(pcs, bs)])
        xp = (C.c_void_p * n)(*[_dev(x, p.prob.n_unknowns, "x") for p, x in zip(pcs, outs)])
        L.check(_lib().shipwave_precond_apply_batched(n, hp, bp, xp, _stream()))
        return outs

    def close(self):
        if self.handle:
            torch.cuda.current_stream().synchronize()
            self.lib.shipwave_precond_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SolveInfo:
    status: int
    newton_iters: int
    gmres_iters: int
    residual_evals: int
    final_norm: float
    time_total_s: float
    time_precond_s: float
    fp32_error: float = -1.0
    linesearch_backtracks: int = 0


def solve_opts(**kw) -> L.SwSolveOpts:
    lib = _lib()
    o = L.SwSolveOpts()
    lib.shipwave_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if k == "weights" and isinstance(v, str):
            v = WEIGHTS[v]
        if k == "spline_bc" and isinstance(v, str):
            v = SPLINE[v]
        if k == "precond":
            v = v.handle if v is not None else None
        setattr(o, k, v)
    return o


INIT = {"flat": 0, "caller": 1, "linear": 2}


def solve(F: float, eps: float, N: int, M: int, x1: float, xN: float, yM: float, *,
          u0=None, init: str | None = None, want_zeta: bool = True, check: bool = True, **opts):
    """Newton-Krylov solve of E(u) = 0; returns (u, zeta or None, SolveInfo).

    Initial guess: u0 if given (init "caller"), else init "flat" (default) or "linear"
    (u_flat - eps P^{-1} s with this solve's preconditioner)."""
    lib = _lib()
    n = 2 * N * M
    o = solve_opts(**opts)
    if u0 is not None:
        u = u0.clone()
        o.init = INIT["caller"]
    else:
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        o.init = INIT[init or "flat"]
        if o.init == INIT["caller"]:
            raise ValueError("init 'caller' needs u0")
    z = torch.empty(N * M, dtype=torch.float64, device=u.device) if want_zeta else None
    mesh = L.SwMesh(N, M)
    dom = L.SwDomain(x1, xN, yM)
    info = L.SwSolveInfo()
    rc = lib.shipwave_solve(float(F), float(eps), C.byref(mesh), C.byref(dom), C.byref(o),
                            _dev(u, n, "u"), z.data_ptr() if z is not None else None,
                            C.byref(info), _stream())
    si = SolveInfo(info.status, info.newton_iters, info.gmres_iters, info.residual_evals,
                   info.final_norm, info.time_total_s, info.time_precond_s, info.fp32_error,
                   info.linesearch_backtracks)
    if check and rc not in (0, -4):
        L.check(rc)
    return u, z, si


@dataclass
class Result:
    status: int
    newton_iters: int
    gmres_iters: int
    residual_evals: int
    used_fallback: int
    final_norm: float
    t_submit_s: float
    t_admit_s: float
    t_done_s: float
    zeta: object = None
    fp32_error: float = -1.0


class Server:
    """Continuous-batching solve server (one worker thread and stream on the GPU).

    q_blocks < 0 lets the server choose the preconditioner band by mesh (5 for N <= 200,
    8 beyond)."""

    def __init__(self, hbm_budget_bytes: float = 8e9, max_slots: int = 16,
                 precision: str = "fp32", fallback_fp64: bool = True, tol: float = 1e-10,
                 q_blocks: int = -1):
        self.lib = _lib()
        o = L.SwServerOpts()
        o.hbm_budget_bytes = float(hbm_budget_bytes)
        o.max_slots = int(max_slots)
        o.fallback_fp64 = 1 if fallback_fp64 else 0
        o.tol = float(tol)
        o.q_blocks = int(q_blocks)
        o.precision = PRECISION[precision]
        h = C.c_void_p()
        L.check(self.lib.shipwave_server_create(C.byref(o), C.byref(h)))
        self.opts = o
        self.handle = h
        self.meshes = {}

    @staticmethod
    def _request(F, eps, N, M, x1, xN, yM):
        r = L.SwRequest()
        r.mesh.N, r.mesh.M = N, M
        r.domain.x1, r.domain.xN, r.domain.yM = x1, xN, yM
        r.F, r.eps = F, eps
        return r

    def request_bytes(self, F, eps, N, M, x1, xN, yM) -> int:
        """Device bytes the server charges for this request (state + preconditioner)."""
        b = C.c_uint64()
        L.check(self.lib.shipwave_server_request_bytes(
            C.byref(self.opts), C.byref(self._request(F, eps, N, M, x1, xN, yM)), C.byref(b)))
        return b.value

    def submit(self, F, eps, N, M, x1, xN, yM) -> int:
        r = self._request(F, eps, N, M, x1, xN, yM)
        t = C.c_uint64()
        L.check(self.lib.shipwave_server_submit(self.handle, C.byref(r), C.byref(t)))
        self.meshes[t.value] = N * M
        return t.value

    def poll(self, ticket: int):
        """Result (with zeta as a numpy array) or None while pending."""
        import numpy as np
        res = L.SwResult()
        z = np.empty(self.meshes[ticket], dtype=np.float64)
        rc = self.lib.shipwave_server_poll(self.handle, C.c_uint64(ticket), C.byref(res),
                                           z.ctypes.data_as(C.c_void_p))
        if rc == -6:
            return None
        L.check(rc)
        return Result(res.status, res.newton_iters, res.gmres_iters, res.residual_evals,
                      res.used_fallback, res.final_norm, res.t_submit_s, res.t_admit_s,
                      res.t_done_s, z, res.fp32_error)

    def drain(self):
        L.check(self.lib.shipwave_server_drain(self.handle))

    def close(self):
        if self.handle:
            self.lib.shipwave_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
