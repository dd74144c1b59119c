#!/usr/bin/env python3
"""Benchmark of the MI355X ship-wave Newton-Krylov path.

One step = one complete FP64 Jacobian-free Newton-Krylov solve of the 181 x 61
workload (x in [-16, 8], y in [0, 12], eps = 0.1, F = 0.7) from the flat
surface to ||E||_inf <= 1e-10, including the set-up of the banded
linear-Jacobian preconditioner (block half-bandwidth q, default 4).  Inputs
are synthetic (the flat state), device-resident before timing starts.

Printed on one JSON line:
  value          solves/s over the timed steps (whole job, one GPU)
  roofline       the all-pairs residual kernel, timed live with HIP events on
                 its launch stream: 48 algorithmic flops per (collocation,
                 grid) pair against the FP64 vector peak of the MI355X; HBM
                 traffic and the instruction-counted FP64 rate come from the
                 committed rocprofv3 counter summaries in profiles/ (null once
                 the kernel source differs from the one they were taken on)
  cpu_baseline   the FP64 CPU oracle on a bounded sample of the same workload
  extra          residual throughput on the 16-state batch (FP64, FP32-Kahan),
                 solve with a prebuilt preconditioner, mixed-precision solve,
                 iteration counts
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 48          # algorithmic flop-equivalents per pair (FMA = 2, rsqrt = 1)
FP64_VECTOR_PEAK_TFLOPS = 78.6
PAPER_TABLE1_181x61_GPU_S = 0.18   # M2090 function evaluation, eps = 1, F = 0.7 (Table 1)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--q", type=int, default=5,
                    help="preconditioner block half-bandwidth (serving: < 0 chooses by mesh)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--serving", action="store_true",
                    help="serving workload: Poisson arrivals of mixed solves (prints its own line)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--residuals", action="store_true",
                    help="residual throughput on configs 1-4, FP64 and FP32-Kahan (own line)")
    ap.add_argument("--workloads", action="store_true",
                    help="config-3 solves (F x eps grid, FP64 and mixed) and the config-4 "
                         "eps continuation (own line)")
    return ap.parse_args()


def _counter_record(name):
    """A committed counter summary for the all-pairs kernel, or None when the
    kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_1403_5044_amd", "csrc", "residual.hip")
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    return rec if rec.get("source_sha256") == digest else None


def measured_traffic():
    """HBM bytes per all-pairs launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    rec = _counter_record("k_pairs_f64_181x61_hbm_counters.json")
    return rec["traffic_bytes_per_launch"] if rec else None


def counted_rate(avg_ms):
    """FP64 rate counted by instruction type (64 lanes x (2 FMA + MUL + ADD + TRANS)
    per wave instruction, from SQ_INSTS_VALU_*_F64) over the live launch time."""
    rec = _counter_record("k_pairs_f64_181x61_fp64_inst_counters.json")
    if not rec or not avg_ms:
        return None
    tf = rec["counted_flops_per_dispatch"] / (avg_ms * 1e-3) / 1e12
    return {"tflops": tf, "frac": tf / FP64_VECTOR_PEAK_TFLOPS,
            "flops_per_pair": rec["counted_flops_per_pair"]}


def cpu_baseline(cfg, evals_per_solve):
    """Time the oracle's FP64 residual on config-2 states: the full E(u) of one
    perturbed linear-solution state, then scale by the residual evaluations one
    GPU solve needed (Krylov, preconditioner and line-search work are left
    out, which favours the CPU)."""
    import numpy as np
    from oracle import Problem as OProblem
    from oracle.equations import residual as oresidual
    from paper_1403_5044_amd import inputs
    op = OProblem(cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"], F=cfg["F"], eps=cfg["eps"])
    u = inputs.config2_batch(1)[0]
    t0 = time.perf_counter()
    E = oresidual(op, u)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(E))
    pairs = (op.N - 1) * op.M * op.N * op.M
    per_solve = dt * evals_per_solve
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"one full FP64 oracle residual E(u) on 181x61 (numpy, single thread): "
                       f"{dt:.2f} s = {pairs / dt:.3e} pairs/s; scaled by the {evals_per_solve} "
                       f"residual evaluations of one GPU solve")}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.serving:
        return serving(args)
    if args.residuals:
        return residuals()
    if args.workloads:
        return workloads()
    import torch
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()  # fails loudly if the HIP library is not built
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    cfg = inputs.CONFIG2
    N, M = cfg["N"], cfg["M"]
    solve_kw = dict(q_blocks=args.q, tol=1e-10)

    def one_solve(**kw):
        kk = dict(solve_kw)
        kk.update(kw)
        return api.solve(cfg["F"], cfg["eps"], N, M, cfg["x1"], cfg["xN"], cfg["yM"], **kk)

    for _ in range(args.warmup):
        one_solve()
    torch.cuda.synchronize()
    api.profile_enable(True)
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        _, _, info = one_solve()
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kms, pairs = api.profile_read()
    api.profile_enable(False)
    for i, info in enumerate(infos):
        print(f"step {i}: {info}", file=sys.stderr, flush=True)
        if info.status != 0:
            print("solve did not converge", file=sys.stderr)
            sys.exit(1)
    dt = t1 - t0
    value = args.steps / dt
    avg_ms = kms / max(launches, 1)
    flops_per_launch = FLOP_PER_PAIR * pairs / max(launches, 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": measured_traffic(),
                "kernel": "k_pairs_f64 (all-pairs boundary-integral sum)",
                "launches": launches, "avg_launch_ms": avg_ms,
                "flop_per_launch": flops_per_launch, "counted": counted_rate(avg_ms)}
    extra = {"newton_iters": infos[-1].newton_iters, "gmres_iters": infos[-1].gmres_iters,
             "residual_evals": infos[-1].residual_evals,
             "precond_build_s": infos[-1].time_precond_s,
             "pair_kernel_share_of_step": kms * 1e-3 / dt}
    if not args.no_extra:
        extra.update(extra_measurements(api, inputs, cfg, one_solve, args.q))
    out = {
        "metric": "JFNK solves/s & pair-interactions/s (frac FP64 peak); p50/p99 solve latency",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"FP64 JFNK solve from the flat surface, mesh {N}x{M}, "
                                f"x in [{cfg['x1']}, {cfg['xN']}], y in [0, {cfg['yM']}], "
                                f"eps {cfg['eps']}, F {cfg['F']}, tol 1e-10, preconditioner "
                                f"q={args.q} built inside each step"),
                   "unknowns": 2 * N * M, "pairs_per_residual": (N - 1) * M * N * M},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, infos[-1].residual_evals)
    out["extra"] = extra
    print(json.dumps(out), flush=True)


def extra_measurements(api, inputs, cfg, one_solve, q):
    import torch
    res = {}
    p = api.Problem(**cfg)
    batch = [torch.tensor(u, device="cuda") for u in inputs.config2_batch(16)]
    outs = [torch.empty_like(b) for b in batch]
    for prec in ("fp64", "fp32"):
        pp = p.with_(precision=prec)
        for u, e in zip(batch, outs):
            api.residual(pp, u, out=e)
        torch.cuda.synchronize()
        reps = 3
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            for u, o in zip(batch, outs):
                api.residual(pp, u, out=o)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / (reps * len(batch))
        res[f"batch16_{prec}_residual_ms"] = ms
        res[f"batch16_{prec}_pairs_per_s"] = p.pairs / (ms * 1e-3)
        res[f"batch16_{prec}_residuals_per_s"] = 1e3 / ms
    res["paper_table1_181x61_gpu_eval_s"] = PAPER_TABLE1_181x61_GPU_S
    # solve with a prebuilt preconditioner (reused across solves of one mesh and F)
    P = api.Preconditioner(p, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = one_solve(precond=P)
    torch.cuda.synchronize()
    res["solve_prebuilt_precond_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, _, infom = one_solve(precond=P, precision="fp32")
    torch.cuda.synchronize()
    res["solve_mixed_prebuilt_precond_s"] = time.perf_counter() - t0
    res["solve_mixed_iters"] = [infom.newton_iters, infom.gmres_iters, infom.residual_evals]
    P.close()
    return res


def calibrate_copy():
    """Three copies of 1 GiB between device buffers (torch's copy kernel): the
    reference dispatch for scaling FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "dispatches": 3}))


def serving(args):
    """Serving workload: requests with Poisson arrivals, meshes uniform over
    {61x21, 121x41, 181x61, 241x81} on x in [-16, 8], y in [0, 12],
    F ~ U[0.5, 1.0], eps ~ U[0.05, 0.4] (seed 0).  First a closed-loop run
    (all requests at once) measures the mixed-precision capacity; the arrival
    rate is set to 80% of it.  Then the same arrival sequence is served in
    mixed precision (FP32-Kahan inner JVPs, FP64 fallback) and in plain FP64,
    each by a warmed server (preconditioners cached per mesh and F bucket)."""
    import numpy as np
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()
    dom = inputs.SERVING_DOMAIN

    def run(srv, reqs, rate=None):
        t0 = time.perf_counter()
        tickets = []
        for (ta, N, M, F, eps) in reqs:
            if rate is not None:
                delay = ta - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            tickets.append(srv.submit(F, eps, N, M, dom["x1"], dom["xN"], dom["yM"]))
        srv.drain()
        wall = time.perf_counter() - t0
        res = [srv.poll(t) for t in tickets]
        lat = np.array([r.t_done_s - r.t_submit_s for r in res])
        ok = sum(1 for r in res if r.status == 0)
        return {"requests": len(res), "converged": ok,
                "fallbacks": sum(r.used_fallback for r in res),
                "wall_s": wall, "solves_per_s": len(res) / wall,
                "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_newton": float(np.mean([r.newton_iters for r in res])),
                "mean_gmres": float(np.mean([r.gmres_iters for r in res])),
                "mean_evals": float(np.mean([r.residual_evals for r in res]))}

    base = inputs.serving_requests(args.requests, 1.0, 0)
    out = {}
    servers = {}
    for prec in ("fp32", "fp64"):
        servers[prec] = api.Server(hbm_budget_bytes=64e9, max_slots=32, precision=prec,
                                   fallback_fp64=True, q_blocks=-1)
        out[f"closed_loop_{prec}"] = run(servers[prec], base)   # warms the caches
    capacity = out["closed_loop_fp32"]["solves_per_s"]
    rate = 0.8 * capacity
    reqs = inputs.serving_requests(args.requests, rate, 0)
    for prec in ("fp32", "fp64"):
        out[f"poisson_{prec}"] = run(servers[prec], reqs, rate=rate)
        servers[prec].close()
    line = {"metric": "JFNK solves/s & pair-interactions/s (frac FP64 peak); p50/p99 solve latency",
            "value": out["poisson_fp32"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.requests, "warmup": args.requests, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": (f"serving: {args.requests} requests, Poisson arrivals at "
                                    f"{rate:.2f}/s (80% of closed-loop mixed capacity), meshes "
                                    f"61x21/121x41/181x61/241x81, F~U[0.5,1], eps~U[0.05,0.4], "
                                    f"seed 0, q by mesh (5 for N <= 200, 8 beyond)")},
            "p50_latency_s": out["poisson_fp32"]["p50_latency_s"],
            "p99_latency_s": out["poisson_fp32"]["p99_latency_s"],
            "arrival_rate_per_s": rate, "runs": out}
    print(json.dumps(line), flush=True)


def _line(value, unit, workload, extra, dtype="f64", higher=True):
    return {"metric": "JFNK solves/s & pair-interactions/s (frac FP64 peak); p50/p99 solve latency",
            "value": value, "unit": unit, "n_gpus": 1, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": {"workload": workload}, **extra}


def residuals():
    """Whole-residual throughput (prelude, pair sum and finish) on configs 1-4 from a
    smooth synthetic state, each precision timed over repeated calls with HIP events."""
    import torch
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()
    rows = {}
    for name, cfg, reps in (("config1", inputs.CONFIG1, 50), ("config2", inputs.CONFIG2, 50),
                            ("config3", inputs.CONFIG3, 10), ("config4", inputs.CONFIG4, 3)):
        for prec in ("fp64", "fp32"):
            p = api.Problem(**cfg, precision=prec)
            u = torch.tensor(inputs.smooth_state(p.N, p.M, 0.02, 1), device="cuda")
            E = api.residual(p, u)
            torch.cuda.synchronize()
            s = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(reps):
                api.residual(p, u, out=E)
            e.record()
            torch.cuda.synchronize()
            ms = s.elapsed_time(e) / reps
            rows[f"{name}_{prec}"] = {
                "mesh": f"{p.N}x{p.M}", "ms_per_residual": ms, "pairs_per_s": p.pairs / ms * 1e3,
                "algorithmic_tflops": FLOP_PER_PAIR * p.pairs / ms * 1e-9,
                "frac_of_peak": FLOP_PER_PAIR * p.pairs / ms * 1e-9 /
                (FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else 2 * FP64_VECTOR_PEAK_TFLOPS)}
    print(json.dumps(_line(rows["config4_fp64"]["pairs_per_s"], "pairs/s",
                           "whole residual E(u) on configs 1-4 (smooth state), FP64 and FP32-Kahan",
                           {"rows": rows})), flush=True)


def workloads():
    """Config 3: 361x121 on the paper's domain, F in {0.5, 0.7, 1.0} x eps in {0.1, 0.3},
    each solved in FP64 and in mixed precision with one preconditioner per F (q = 8).
    Config 4: 721x241, F = 0.7, eps continued 0.1 -> 0.5 in mixed precision (q = 8), with
    FP64 solves at the first and last eps for comparison."""
    import torch
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()
    kw = dict(tol=1e-10, max_gmres=600, gmres_restart=60, max_newton=20)

    def timed(F, eps, cfg, prec, P, u0=None):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, z, info = api.solve(F, eps, cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"],
                               precision=prec, precond=P, u0=u0, **kw)
        torch.cuda.synchronize()
        return u, z, {"status": info.status, "newton": info.newton_iters,
                      "gmres": info.gmres_iters, "evals": info.residual_evals,
                      "final_norm": info.final_norm, "s": time.perf_counter() - t0,
                      "zeta_max": z.max().item()}

    def build(cfg, q):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = api.Preconditioner(api.Problem(**cfg), q)
        torch.cuda.synchronize()
        return P, time.perf_counter() - t0

    out = {"config3": [], "config4": []}
    c3 = inputs.CONFIG3
    for F in inputs.CONFIG3_F:
        P, tb = build(dict(c3, F=F), 8)
        for eps in inputs.CONFIG3_EPS:
            _, z64, r64 = timed(F, eps, c3, "fp64", P)
            _, z32, r32 = timed(F, eps, c3, "fp32", P)
            out["config3"].append({"F": F, "eps": eps, "build_s": tb, "fp64": r64, "mixed": r32,
                                   "zeta_mixed_vs_fp64": (z64 - z32).abs().max().item()})
            print(f"config3 F={F} eps={eps}: fp64 {r64['s']:.2f}s mixed {r32['s']:.2f}s",
                  file=sys.stderr, flush=True)
        P.close()
    c4 = inputs.CONFIG4
    P, tb = build(c4, 8)
    out["config4_build_s"] = tb
    u = None
    for eps in inputs.CONFIG4_EPS:
        um, zm, rm = timed(c4["F"], eps, c4, "fp32", P, u)
        rec = {"eps": eps, "mixed": rm}
        if eps in (inputs.CONFIG4_EPS[0], inputs.CONFIG4_EPS[-1]):
            _, z64, r64 = timed(c4["F"], eps, c4, "fp64", P, u)
            rec["fp64"] = r64
            rec["zeta_mixed_vs_fp64"] = (z64 - zm).abs().max().item()
        out["config4"].append(rec)
        print(f"config4 eps={eps}: mixed {rm['s']:.2f}s status {rm['status']}", file=sys.stderr,
              flush=True)
        if rm["status"] != 0:
            break
        u = um
    P.close()
    n = len(out["config4"])
    total = sum(r["mixed"]["s"] for r in out["config4"])
    print(json.dumps(_line(n / total, "solves/s",
                           "config-4 eps continuation 0.1..0.5 (721x241, mixed, q=8); "
                           "config-3 F x eps grid in FP64 and mixed (361x121, q=8)",
                           {"runs": out}, dtype="f32+f64")), flush=True)


if __name__ == "__main__":
    main()
