"""Batched residual and the continuous-batching server on the GPU."""
import time

import numpy as np
import pytest
import torch

from oracle import flat_state as oflat
from oracle.equations import zeta_grid
from oracle.solve import newton
from paper_1403_5044_amd import api, inputs

from gpu_common import dev, gprob, host, log, oprob

pytestmark = pytest.mark.gpu

DOM = inputs.SERVING_DOMAIN


def test_batched_residual_is_bitwise_the_single_residual():
    probs = [gprob(inputs.W31X11),
             api.Problem(61, 21, **DOM, F=0.6, eps=0.2, precision="fp32"),
             api.Problem(121, 41, **DOM, F=0.9, eps=0.3),
             api.Problem(9, 5, -3.0, 3.0, 2.0, F=0.7, eps=0.3),
             api.Problem(181, 61, **DOM, F=0.7, eps=0.1, precision="fp32"),
             api.Problem(40, 9, -6.0, 5.0, 4.0, F=0.9, eps=0.2, weights="trapezoid")]
    us = [dev(inputs.smooth_state(p.N, p.M, 0.05, i)) for i, p in enumerate(probs)]
    single = [host(api.residual(p, u)) for p, u in zip(probs, us)]
    batched = [host(e) for e in api.residual_batched(probs, us)]
    for p, a, b in zip(probs, single, batched):
        assert np.array_equal(a, b), (p.N, p.M, p.precision)


def _serve(reqs, **kw):
    srv = api.Server(**kw)
    tickets = [srv.submit(*r) for r in reqs]
    srv.drain()
    res = [srv.poll(t) for t in tickets]
    srv.close()
    return res


REQS = [(0.7, 0.05, 31, 11, -8.0, 8.0, 8.0),
        (0.6, 0.2, 61, 21, -16.0, 8.0, 12.0),
        (0.9, 0.1, 61, 21, -16.0, 8.0, 12.0),
        (0.55, 0.3, 121, 41, -16.0, 8.0, 12.0),
        (0.8, 0.15, 31, 11, -8.0, 8.0, 8.0),
        (1.0, 0.4, 61, 21, -16.0, 8.0, 12.0)]


def test_server_fp64_results_match_the_oracle_root():
    res = _serve(REQS[:2], precision="fp64", max_slots=4)
    for r, req in zip(res, REQS[:2]):
        log(f"server fp64 {req[2]}x{req[3]}: {r.status} newton {r.newton_iters} gmres "
            f"{r.gmres_iters} evals {r.residual_evals} latency {r.t_done_s - r.t_submit_s:.3f}s")
        assert r.status == 0
        F, eps, N, M, x1, xN, yM = req
        op = oprob(api.Problem(N, M, x1, xN, yM, F=F, eps=eps))
        uo, info = newton(op, oflat(op), tol=1e-12)
        assert info.converged
        err = np.abs(r.zeta - zeta_grid(op, uo).ravel()).max()
        log(f"  zeta err vs oracle {err:.2e}")
        assert err <= 1e-8


def test_server_result_is_identical_alone_and_in_a_mix():
    alone = _serve([REQS[3]], precision="fp32", max_slots=8)[0]
    mix = _serve(REQS[:3] + [REQS[3]] + REQS[4:], precision="fp32", max_slots=8)
    inmix = mix[3]
    assert alone.status == 0 and inmix.status == 0
    assert np.array_equal(alone.zeta, inmix.zeta)
    assert (alone.newton_iters, alone.gmres_iters) == (inmix.newton_iters, inmix.gmres_iters)
    for r in mix:
        assert r.status == 0


def test_server_result_is_bitwise_the_direct_solve():
    """The server runs each Krylov step's preconditioner apply, shifted state, Gram-Schmidt
    passes and norm batched across the active solves. For requests whose F lies on the
    grid of the server's preconditioner cache (so that its preconditioner is the one a
    direct solve builds) the served zeta and iteration counts equal the direct solve's bit
    for bit, in FP64 and mixed precision, with all requests in one mix."""
    dom = tuple(DOM.values())
    reqs = [(0.75, 0.2, 61, 21, *dom), (0.5, 0.3, 121, 41, *dom),
            (1.0, 0.1, 31, 11, -8.0, 8.0, 8.0), (0.625, 0.15, 61, 21, *dom)]
    for r in reqs:
        assert round(r[0] / 0.025) * 0.025 == r[0]
    for prec in ("fp64", "fp32"):
        res = _serve(reqs, precision=prec, max_slots=8)
        for r, (F, eps, N, M, x1, xN, yM) in zip(res, reqs):
            assert r.status == 0 and r.used_fallback == 0
            _, z, info = api.solve(F, eps, N, M, x1, xN, yM, precision=prec, q_blocks=5)
            assert info.status == 0
            log(f"{prec} {N}x{M} F={F}: server newton {r.newton_iters} gmres {r.gmres_iters}, "
                f"direct {info.newton_iters} / {info.gmres_iters}, "
                f"max |dzeta| {np.abs(host(z) - r.zeta).max():.1e}")
            assert (r.newton_iters, r.gmres_iters) == (info.newton_iters, info.gmres_iters)
            assert np.array_equal(host(z), r.zeta)


def test_server_with_more_solves_than_one_batched_launch_takes():
    """40 solves submitted at once (a batched Krylov launch or a batch of applies takes
    up to 32 solves), with requests sharing cached preconditioners (their applies go in
    separate batches): every served zeta equals its direct solve bit for bit."""
    dom = tuple(DOM.values())
    reqs = []
    for k in range(40):
        N, M = (31, 11) if k % 2 else (61, 21)
        reqs.append((0.025 * (20 + k % 9), 0.05 + 0.01 * k, N, M, *dom))
        assert round(reqs[-1][0] / 0.025) * 0.025 == reqs[-1][0]
    res = _serve(reqs, precision="fp64", max_slots=48, hbm_budget_bytes=16e9)
    for r, (F, eps, N, M, x1, xN, yM) in zip(res, reqs):
        assert r.status == 0
        _, z, info = api.solve(F, eps, N, M, x1, xN, yM, q_blocks=5)
        assert info.status == 0
        assert (r.newton_iters, r.gmres_iters) == (info.newton_iters, info.gmres_iters)
        assert np.array_equal(host(z), r.zeta), (N, M, F, eps)
    log(f"40 served solves equal their direct solves; mean latency "
        f"{np.mean([r.t_done_s - r.t_submit_s for r in res]) * 1e3:.1f} ms")


def test_server_mixed_precision_matches_fp64_within_bound():
    r64 = _serve(REQS, precision="fp64", max_slots=8)
    r32 = _serve(REQS, precision="fp32", max_slots=8)
    for a, b, req in zip(r64, r32, REQS):
        assert a.status == 0 and b.status == 0
        err = np.abs(a.zeta - b.zeta).max()
        log(f"{req[2]}x{req[3]} F={req[0]} eps={req[1]}: mixed vs fp64 zeta {err:.2e}, "
            f"fallback {b.used_fallback}")
        assert err <= 1e-6


def test_server_admission_by_memory_budget():
    # budget below any request: rejected with SW_ENOMEM
    res = _serve(REQS[:2], precision="fp64", hbm_budget_bytes=1e5)
    assert all(r.status == -2 for r in res)
    # budget for one 61x21 request at a time: all complete, one after another
    probe = api.Server(precision="fp64")
    one = 1.5 * max(probe.request_bytes(*REQS[1]), probe.request_bytes(*REQS[2]))
    probe.close()
    res = _serve([REQS[1], REQS[2]], precision="fp64", hbm_budget_bytes=one, max_slots=8)
    assert all(r.status == 0 for r in res)
    assert res[1].t_admit_s >= res[0].t_done_s - 1e-6


def test_server_rejects_invalid_requests():
    res = _serve([(0.7, 0.1, 3, 11, -8.0, 8.0, 8.0), REQS[0]], precision="fp64")
    assert res[0].status == -1 and res[1].status == 0


def test_server_large_serving_meshes_satisfy_the_oracle():
    """The two larger serving meshes (181x61 and 241x81, the server's q = 5 and 8) in one
    mix with the smaller ones: every result converges, mixed precision agrees with FP64
    within 1e-6, and the FP64 roots satisfy the oracle's E on sampled rows to 1e-9 (each
    E2 row a full sum over the grid)."""
    from oracle import Problem as OProblem
    from oracle.equations import residual_rows
    reqs = [(0.65, 0.25, 241, 81, *DOM.values()),
            (0.85, 0.15, 181, 61, *DOM.values()),
            (0.75, 0.35, 121, 41, *DOM.values()),
            (0.95, 0.1, 61, 21, *DOM.values())]
    r64 = _serve(reqs, precision="fp64", max_slots=8, hbm_budget_bytes=64e9)
    r32 = _serve(reqs, precision="fp32", max_slots=8, hbm_budget_bytes=64e9)
    rng = np.random.default_rng(3)
    for a, b, (F, eps, N, M, x1, xN, yM) in zip(r64, r32, reqs):
        assert a.status == 0 and b.status == 0
        dz = np.abs(a.zeta - b.zeta).max()
        log(f"server {N}x{M} F={F} eps={eps}: fp64 newton {a.newton_iters} gmres "
            f"{a.gmres_iters}; mixed vs fp64 zeta {dz:.2e}")
        assert dz <= 1e-6
        # the server returns zeta; the state comes from a direct solve of the same request
        # (tol 1e-12), whose zeta must agree with the server's (tol 1e-10) to within
        # 1e-7, a thousand times the server's residual tolerance
        u, z, info = api.solve(F, eps, N, M, x1, xN, yM, tol=1e-12, max_gmres=600,
                               gmres_restart=60)
        assert info.status == 0
        dd = np.abs(host(z) - a.zeta).max()
        log(f"  server vs direct solve zeta {dd:.2e}")
        assert dd <= 1e-7
        op = OProblem(N, M, x1, xN, yM, F=F, eps=eps)
        NM = N * M
        e2 = NM + rng.integers(0, M, 8) * N + rng.integers(1, N, 8)
        rows = np.unique(np.concatenate([np.arange(0, NM, 13), e2]))
        E, _ = residual_rows(op, host(u), rows)
        log(f"  oracle |E| at the direct solve's root on {rows.size} rows: {np.abs(E).max():.2e}")
        assert np.abs(E).max() <= 1e-9
