"""Solver paths other than the plain converging solve, through the C ABI:

  * the linear-solution initial guess against the oracle's discrete linear solution;
  * the FP32 error estimate of sw_solve_info against a direct computation;
  * failure paths forced from the host (a NaN written into one residual output after
    its kernels, shipwave_debug_inject_nonfinite): line-search backtracking,
    SW_ENONFINITE, SW_ENOCONV and the server's FP64 fallback.  Every kernel runs to
    completion; only the host logic sees the non-finite value.
"""
import numpy as np
import pytest
import torch

from oracle import Problem as OProblem
from oracle import flat_state as oflat
from oracle import linear as OL
from oracle.equations import zeta_grid
from oracle.solve import newton
from paper_1403_5044_amd import api, inputs

from gpu_common import dev, gprob, host, log, oprob

pytestmark = pytest.mark.gpu

C1 = inputs.W31X11
ARGS1 = (C1["F"], C1["eps"], C1["N"], C1["M"], C1["x1"], C1["xN"], C1["yM"])


@pytest.fixture
def inject():
    yield api.debug_inject_nonfinite
    api.debug_inject_nonfinite(0, 0)


def _oracle_zeta(p):
    op = oprob(p)
    u, info = newton(op, oflat(op), tol=1e-12)
    assert info.converged
    return zeta_grid(op, u).ravel()


@pytest.mark.parametrize("cfg", [C1, dict(N=41, M=13, x1=-8.0, xN=8.0, yM=6.0, F=0.9,
                                          eps=0.3)])
def test_linear_initial_guess_is_the_discrete_linear_solution(cfg):
    """init = 2 with the full linear preconditioner (q = M - 1): the state handed to the
    first evaluation (returned as is under a tolerance it already meets) equals the
    oracle's linear solution u_flat - eps J_lin^{-1} s; the solve from it reaches the
    same root as the solve from the flat surface."""
    p = gprob(cfg)
    args = (p.F, p.eps, p.N, p.M, p.x1, p.xN, p.yM)
    op = oprob(p)
    ul = OL.linear_solution(op)
    u0, _, i0 = api.solve(*args, init="linear", q_blocks=p.M - 1, tol=1e3)
    assert i0.status == 0 and i0.newton_iters == 0
    d = host(u0) - ul
    rel = np.abs(d).max() / np.abs(ul - oflat(op)).max()
    log(f"{p.N}x{p.M}: linear initial guess vs oracle, max rel err {rel:.2e}")
    assert rel <= 1e-8
    ua, za, ia = api.solve(*args, init="linear", q_blocks=p.M - 1, tol=1e-11)
    ub, zb, ib = api.solve(*args, q_blocks=p.M - 1, tol=1e-11)
    log(f"  from linear: {ia}\n  from flat:   {ib}")
    assert ia.status == 0 and ib.status == 0
    assert np.abs(host(za) - _oracle_zeta(p)).max() <= 1e-8
    assert np.abs(host(za) - host(zb)).max() <= 1e-9


def test_fp32_error_estimate_matches_a_direct_computation():
    p = gprob(C1)
    for prec in ("fp64", "fp32"):
        u, _, info = api.solve(*ARGS1, precision=prec, tol=1e-11)
        assert info.status == 0
        E64 = api.residual(p, u)
        E32 = api.residual(p.with_(precision="fp32"), u)
        want = ((E32 - E64).abs().max() / max(1.0, E64.abs().max().item())).item()
        log(f"{prec}: fp32_error {info.fp32_error:.3e}, direct {want:.3e}")
        assert info.fp32_error == pytest.approx(want, rel=1e-12)
        assert 0.0 < info.fp32_error <= 1e-5


def test_enoconv_keeps_the_best_iterate():
    p = gprob(C1)
    E0 = np.abs(host(api.residual(p, dev(inputs.flat_state(p.N, p.M))))).max()
    u, _, info = api.solve(*ARGS1, max_newton=1, tol=1e-15)
    log(f"max_newton 1: {info}")
    assert info.status == -4 and info.newton_iters == 1
    assert np.all(np.isfinite(host(u)))
    En = np.abs(host(api.residual(p, u))).max()
    assert En == info.final_norm and En < E0
    assert info.fp32_error > 0.0


def test_nonfinite_initial_residual_is_reported(inject):
    inject(1, 1)
    _, _, info = api.solve(*ARGS1, check=False)
    log(f"NaN in E(u0): {info}")
    assert info.status == -5 and info.newton_iters == 0 and info.fp32_error == -1.0


def test_nonfinite_jvp_is_reported(inject):
    inject(4, 3)
    _, _, info = api.solve(*ARGS1, check=False)
    log(f"NaN in the third FP64 JVP: {info}")
    assert info.status == -5


def test_line_search_backtracks_past_a_nonfinite_trial(inject):
    """The first trial point's residual is made non-finite: lambda halves, the half step
    is accepted, and Newton still reaches the oracle's root."""
    p = gprob(C1)
    inject(2, 1)
    _, z, info = api.solve(*ARGS1, tol=1e-11)
    log(f"NaN at the first line-search trial: {info}")
    assert info.status == 0 and info.linesearch_backtracks == 1
    assert np.abs(host(z) - _oracle_zeta(p)).max() <= 1e-8
    api.debug_inject_nonfinite(0, 0)
    _, _, clean = api.solve(*ARGS1, tol=1e-11)
    assert clean.linesearch_backtracks == 0
    assert info.newton_iters >= clean.newton_iters


@pytest.mark.parametrize("fallback", [True, False])
def test_server_falls_back_to_fp64(inject, fallback):
    """A mixed-precision solve whose second FP32 JVP is non-finite fails with
    SW_ENONFINITE; with fallback the server re-solves it in FP64 (whose JVPs are not
    touched) and the result matches the oracle root."""
    p = gprob(C1)
    inject(8, 2)
    srv = api.Server(precision="fp32", fallback_fp64=fallback, max_slots=4)
    t = srv.submit(*ARGS1)
    srv.drain()
    r = srv.poll(t)
    srv.close()
    log(f"fallback={fallback}: status {r.status}, used_fallback {r.used_fallback}, "
        f"fp32_error {r.fp32_error:.2e}")
    if fallback:
        assert r.status == 0 and r.used_fallback == 1
        assert np.abs(r.zeta - _oracle_zeta(p)).max() <= 1e-8
        assert 0.0 < r.fp32_error <= 1e-5
    else:
        assert r.status == -5 and r.used_fallback == 0
