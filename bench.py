#!/usr/bin/env python3
"""Benchmark of the MI355X ship-wave Newton-Krylov path.

One step = one complete FP64 Jacobian-free Newton-Krylov solve of the largest
workload, 721 x 241 on the paper's domain (x in [-14, 40], y in [0, 18],
spacing 0.075, eps = 0.1, F = 0.7), from the flat surface to
||E||_inf <= 1e-10, including the set-up of the banded linear-Jacobian
preconditioner (block half-bandwidth q, default 16: a band of 1.2 in y, where
GMRES per Newton step levels off) inside the step.  Inputs are
synthetic (the flat state), device-resident before timing starts.

Printed on one JSON line:
  value          solves/s over the timed steps (whole job, one GPU)
  pair_interactions_per_s
                 pairs per all-pairs launch / its average launch time
  roofline       the all-pairs residual kernel, timed live with HIP events on
                 its launch stream: 48 algorithmic flops per (collocation,
                 grid) pair against the FP64 vector peak of the MI355X; HBM
                 traffic and the instruction-counted FP64 rate come from the
                 committed rocprofv3 counter summaries in profiles/ (null once
                 the kernel source differs from the one they were taken on)
  p50/p99        solve latency of the serving workload (Poisson arrivals,
                 mixed precision; FP64 beside it)
  fp32_error     mixed-precision solve of the same workload: the FP32-Kahan
                 residual against the FP64 oracle on sampled rows, and the
                 solve's own estimate
  cpu_baseline   the FP64 CPU oracle on a bounded sample of the same workload
                 (one thread and all cores), plus an oracle solve of the
                 31 x 11 workload
Other modes print their own line: --serving, --residuals, --workloads,
--table1, --precond-study, --calibrate-copy.
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
METRIC = "JFNK solves/s & pair-interactions/s (frac FP64 peak); p50/p99 solve latency"
# Counter summaries of the all-pairs kernel on the benched workload (profiles/)
HBM_COUNTERS = "k_pairs_f64_721x241_hbm_counters.json"
INST_COUNTERS = "k_pairs_f64_721x241_fp64_inst_counters.json"


def inputs_q_large():
    from paper_1403_5044_amd import inputs
    return inputs.Q_BLOCKS[(inputs.W721X241["N"], inputs.W721X241["M"])]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--q", type=int, default=inputs_q_large(),
                    help="preconditioner block half-bandwidth of the benched solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--serving", action="store_true",
                    help="serving workload: Poisson arrivals of mixed solves (prints its own line)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--out-dir", default=None,
                    help="folder for the detail files of --serving, --table1 and "
                         "--precond-study (per-request times, centrelines, spectra); "
                         "none are written without it")
    ap.add_argument("--serving-rate", type=float, default=None,
                    help="Poisson arrival rate of --serving (default: 80%% of the closed-loop "
                         "mixed capacity)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--residuals", action="store_true",
                    help="residual throughput on the 31x11, 181x61, 361x121 and 721x241 workloads, "
                         "FP64 and FP32-Kahan (own line)")
    ap.add_argument("--workloads", action="store_true",
                    help="361x121 solves (F x eps grid, FP64 and mixed) and the 721x241 "
                         "eps continuation (own line)")
    ap.add_argument("--table1", action="store_true",
                    help="the paper's eps = 1, F = 0.7 workload: per-evaluation times on the "
                         "Table-1 meshes, continuation to eps = 1, centreline, F = 1.4 (own line)")
    ap.add_argument("--precond-study", action="store_true",
                    help="GMRES iterations per Newton step against the block bandwidth (own line)")
    ap.add_argument("--profile-solves", type=int, default=0,
                    help="run only this many benched solves (for rocprofv3) and exit")
    ap.add_argument("--profile-precision", default="fp64", choices=("fp64", "fp32"),
                    help="precision of the --profile-solves / --profile-residuals runs")
    ap.add_argument("--profile-residuals", type=int, default=0,
                    help="run only this many residual evaluations of the benched workload "
                         "on one stream (for rocprofv3 counters) and exit")
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
    rec = _counter_record(HBM_COUNTERS)
    return rec["traffic_bytes_per_launch"] if rec else None


def counted_rate(avg_ms):
    """FP64 rate counted by instruction type (64 lanes x (2 FMA + MUL + ADD + TRANS)
    per wave instruction, from SQ_INSTS_VALU_*_F64) over the live launch time."""
    rec = _counter_record(INST_COUNTERS)
    if not rec or not avg_ms:
        return None
    tf = rec["counted_flops_per_dispatch"] / (avg_ms * 1e-3) / 1e12
    return {"tflops": tf, "frac": tf / FP64_VECTOR_PEAK_TFLOPS,
            "flops_per_pair": rec["counted_flops_per_pair"]}


def _host_description():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def _oracle_rows_worker(args):
    """Time the oracle's all-pairs sum at the given collocation points (one process,
    one thread).  Returns (seconds of the pair sum, seconds of the O(NM) prelude)."""
    cfg, cols = args
    import numpy as np
    from oracle import Problem as OProblem
    from oracle import equations as oeq
    from paper_1403_5044_amd import inputs
    op = OProblem(cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"], F=cfg["F"], eps=cfg["eps"])
    u = inputs.smooth_state(op.N, op.M, 0.02, 1)
    t0 = time.perf_counter()
    geom = oeq._half_geom(op)
    psix, zetax = oeq.unpack(op, u)
    f = oeq.grid_fields(op, geom, psix, zetax)
    oeq.bernoulli(op, f)
    oeq._I_field(geom, f)
    t1 = time.perf_counter()
    S = oeq.pair_sum(geom, f, cols=np.asarray(cols, dtype=np.int64))
    t2 = time.perf_counter()
    assert np.all(np.isfinite(S.ravel()[cols]))
    return t2 - t1, t1 - t0


def cpu_baseline(cfg, evals_per_solve):
    """The FP64 oracle (numpy, as it stands) on a bounded sample of the benched
    workload: its all-pairs sum at sampled collocation points, on one thread and
    then in one single-threaded process per available core, scaled to a whole
    residual and then by the residual evaluations one GPU solve needed (the
    oracle's Krylov, preconditioner and line-search work is left out, which
    favours the CPU).  Also an oracle Newton solve of the 31 x 11 workload."""
    import multiprocessing as mp
    import numpy as np
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    model, avail = _host_description()
    workers = max(1, min(avail or 1, 16))
    ncol = (cfg["N"] - 1) * cfg["M"]
    rng = np.random.default_rng(12345)
    one = rng.choice(ncol, 96, replace=False)
    t_pairs1, t_pre = _oracle_rows_worker((cfg, one))
    per_point1 = t_pairs1 / one.size
    per_res1 = t_pre + per_point1 * ncol
    per_w = 48
    jobs = [(cfg, rng.choice(ncol, per_w, replace=False)) for _ in range(workers)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_rows_worker, jobs)
    wall = time.perf_counter() - t0
    # throughput of all workers together: points done per second of the slowest worker
    slowest = max(r[0] for r in res)
    per_point_all = slowest / per_w / workers
    per_res_all = t_pre + per_point_all * ncol
    # oracle solve of the 31 x 11 workload (dense Newton, exact Jacobian)
    from oracle import Problem as OProblem
    from oracle import flat_state as oflat
    from oracle.solve import newton
    from paper_1403_5044_amd import inputs
    c1 = inputs.W31X11
    op1 = OProblem(c1["N"], c1["M"], c1["x1"], c1["xN"], c1["yM"], F=c1["F"], eps=c1["eps"])
    t0 = time.perf_counter()
    _, oinfo = newton(op1, oflat(op1), tol=1e-10)
    t_c1 = time.perf_counter() - t0
    pairs = ncol * cfg["N"] * cfg["M"]
    return {"value": 1.0 / (per_res_all * evals_per_solve), "unit": "solves/s",
            "cores": workers, "kind": "oracle",
            "sample": (f"FP64 oracle (numpy) all-pairs sum at sampled collocation points of "
                       f"{cfg['N']}x{cfg['M']}: {one.size} points on one thread, then "
                       f"{workers} single-threaded processes x {per_w} points; per residual = "
                       f"O(NM) prelude ({t_pre:.2f} s) + per-point time x {ncol} points; "
                       f"x {evals_per_solve} residual evaluations of one GPU solve"),
            "host_cpu": model, "host_cpus_available": avail,
            "one_thread": {"s_per_residual": per_res1, "pairs_per_s": pairs / per_res1,
                           "solves_per_s": 1.0 / (per_res1 * evals_per_solve)},
            "all_cores": {"threads": workers, "s_per_residual": per_res_all,
                          "pairs_per_s": pairs / per_res_all, "pool_wall_s": wall},
            "oracle_solve_31x11_s": t_c1,
            "oracle_solve_31x11_iters": [oinfo.newton, oinfo.gmres, oinfo.evals]}


def fp32_error_vs_oracle(api, cfg, u, nrows=64):
    """max |E32 - E64_oracle| / max(1, ||E64_oracle||) on every E1 row at stride 37 and
    nrows sampled E2 rows, with E32 the FP32-Kahan residual of the GPU at state u."""
    import numpy as np
    from oracle import Problem as OProblem
    from oracle.equations import residual_rows
    p = api.Problem(**cfg, precision="fp32")
    E32 = api.residual(p, u).cpu().numpy()
    N, M = cfg["N"], cfg["M"]
    NM = N * M
    rng = np.random.default_rng(7)
    e2 = NM + rng.choice(M, nrows) * N + rng.integers(1, N, nrows)
    rows = np.concatenate([np.arange(0, NM, 37), NM + np.arange(M) * N, e2])
    op = OProblem(N, M, cfg["x1"], cfg["xN"], cfg["yM"], F=cfg["F"], eps=cfg["eps"])
    E64, scale = residual_rows(op, u.cpu().numpy(), rows)
    d = np.abs(E32[rows] - E64)
    return {"rows": int(rows.size), "max_abs": float(d.max()),
            "rel": float(d.max() / max(1.0, np.abs(E64).max())),
            "max_over_row_scale": float((d / scale).max())}


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
    if args.table1:
        return table1(args.out_dir)
    if args.precond_study:
        return precond_study(args.out_dir)
    import torch
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()  # fails loudly if the HIP library is not built
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    cfg = inputs.W721X241
    N, M = cfg["N"], cfg["M"]
    solve_kw = dict(q_blocks=args.q, **inputs.LARGE_SOLVE)

    def one_solve(**kw):
        kk = dict(solve_kw)
        kk.update(kw)
        return api.solve(cfg["F"], cfg["eps"], N, M, cfg["x1"], cfg["xN"], cfg["yM"], **kk)

    if args.profile_residuals:
        p = api.Problem(**cfg, precision=args.profile_precision)
        u = torch.tensor(inputs.smooth_state(N, M, 0.02, 1), device="cuda")
        E = api.residual(p, u)
        for i in range(args.profile_residuals):
            api.residual(p, u, out=E)
            torch.cuda.synchronize()
            print(f"profiled residual {i} ({args.profile_precision})", flush=True)
        return
    if args.profile_solves:
        for i in range(args.profile_solves):
            _, _, info = one_solve(precision=args.profile_precision)
            torch.cuda.synchronize()
            print(f"profiled solve {i}: {info}", flush=True)
        return
    for i in range(args.warmup):
        _, _, info = one_solve()
        print(f"warmup {i}: {info}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    api.profile_enable(True)
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        u64, z64, info = one_solve()
        infos.append(info)
        print(f"step {i}: {info}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kms, pairs = api.profile_read()
    api.profile_enable(False)
    if any(i.status != 0 for i in infos):
        print("solve did not converge", file=sys.stderr)
        sys.exit(1)
    dt = t1 - t0
    value = args.steps / dt
    avg_ms = kms / max(launches, 1)
    pairs_per_launch = pairs / max(launches, 1)
    flops_per_launch = FLOP_PER_PAIR * pairs_per_launch
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": measured_traffic(),
                "kernel": "k_pairs_f64 (all-pairs boundary-integral sum)",
                "launches": launches, "avg_launch_ms": avg_ms,
                "flop_per_launch": flops_per_launch, "counted": counted_rate(avg_ms)}
    last = infos[-1]
    extra = {"newton_iters": last.newton_iters, "gmres_iters": last.gmres_iters,
             "residual_evals": last.residual_evals, "final_norm": last.final_norm,
             "precond_build_s": last.time_precond_s,
             "pair_kernel_share_of_step": kms * 1e-3 / dt}
    out = {
        "metric": METRIC,
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"FP64 JFNK solve from the flat surface, mesh {N}x{M}, "
                                f"x in [{cfg['x1']}, {cfg['xN']}], y in [0, {cfg['yM']}] "
                                f"(spacing 0.075), eps {cfg['eps']}, F {cfg['F']}, tol 1e-10, "
                                f"GMRES({solve_kw['gmres_restart']}), preconditioner "
                                f"q={args.q} built inside each step"),
                   "unknowns": 2 * N * M, "pairs_per_residual": (N - 1) * M * N * M},
        "pair_interactions_per_s": pairs_per_launch / (avg_ms * 1e-3),
        "roofline": roofline,
    }
    if not args.no_extra:
        ex = extra_measurements(api, inputs, cfg, one_solve, z64, args)
        out["fp32_error"] = ex.pop("fp32_error")
        srv = ex.pop("serving")
        out["p50_latency_s"] = srv["poisson_fp32"]["p50_latency_s"]
        out["p99_latency_s"] = srv["poisson_fp32"]["p99_latency_s"]
        out["latency"] = {
            "workload": srv["workload"],
            "mixed": {k: srv["poisson_fp32"][k] for k in
                      ("p50_latency_s", "p99_latency_s", "solves_per_s", "converged", "fallbacks")},
            "fp64": {k: srv["poisson_fp64"][k] for k in
                     ("p50_latency_s", "p99_latency_s", "solves_per_s", "converged", "fallbacks")},
            "closed_loop_solves_per_s": {"mixed": srv["closed_loop_fp32"]["solves_per_s"],
                                         "fp64": srv["closed_loop_fp64"]["solves_per_s"]}}
        extra.update(ex)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, last.residual_evals)
    out["extra"] = extra
    print(json.dumps(out), flush=True)


def extra_measurements(api, inputs, cfg, one_solve, z64, args):
    """Residual throughput (this workload and the 16-state 181 x 61 batch), a
    mixed-precision solve of the benched workload with its FP32 error, and the
    serving workload's latency."""
    import torch
    res = {}

    def timed_residuals(p, us, reps):
        outs = [torch.empty_like(u) for u in us]
        for u, e in zip(us, outs):
            api.residual(p, u, out=e)
        torch.cuda.synchronize()
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            for u, o in zip(us, outs):
                api.residual(p, u, out=o)
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / (reps * len(us))

    p4 = api.Problem(**cfg)
    u4 = [torch.tensor(inputs.smooth_state(p4.N, p4.M, 0.02, 1), device="cuda")]
    c2 = api.Problem(**inputs.W181X61)
    batch = [torch.tensor(u, device="cuda") for u in inputs.batch_181x61(16)]
    for prec in ("fp64", "fp32"):
        ms = timed_residuals(p4.with_(precision=prec), u4, 3)
        res[f"residual_{p4.N}x{p4.M}_{prec}_ms"] = ms
        res[f"residual_{p4.N}x{p4.M}_{prec}_pairs_per_s"] = p4.pairs / (ms * 1e-3)
        ms = timed_residuals(c2.with_(precision=prec), batch, 3)
        res[f"batch16_181x61_{prec}_residuals_per_s"] = 1e3 / ms
        res[f"batch16_181x61_{prec}_pairs_per_s"] = c2.pairs / (ms * 1e-3)
    # the same solve in mixed precision (FP32-Kahan inner JVPs, FP64 outer residual)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    um, zm, infom = one_solve(precision="fp32")
    torch.cuda.synchronize()
    res["mixed_solve"] = {"s": time.perf_counter() - t0, "status": infom.status,
                          "newton": infom.newton_iters, "gmres": infom.gmres_iters,
                          "evals": infom.residual_evals, "final_norm": infom.final_norm,
                          "zeta_vs_fp64_solve": (zm - z64).abs().max().item()}
    # the same FP64 solve from the linear-solution initial guess (u_flat - eps P^-1 s with
    # the solve's own preconditioner) instead of the flat surface
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, zl, infol = one_solve(init="linear")
    torch.cuda.synchronize()
    res["linear_init_solve"] = {"s": time.perf_counter() - t0, "status": infol.status,
                                "newton": infol.newton_iters, "gmres": infol.gmres_iters,
                                "evals": infol.residual_evals,
                                "zeta_vs_flat_start": (zl - z64).abs().max().item()}
    err = fp32_error_vs_oracle(api, cfg, um)
    err["solve_estimate"] = infom.fp32_error
    err["what"] = ("FP32-Kahan residual at the mixed-precision root against the FP64 oracle "
                   "on sampled rows (max_abs, rel = / max(1, ||E64||)); solve_estimate = the "
                   "solve's own max|E32 - E64| / max(1, ||E64||) over every entry")
    res["fp32_error"] = err
    print(f"mixed solve: {res['mixed_solve']}; fp32 error {err}", file=sys.stderr, flush=True)
    res["serving"] = serving_runs(api, inputs, args.requests, out_dir=args.out_dir)
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


def serving_runs(api, inputs, nreq, fixed_rate=None, out_dir=None):
    """Serving workload: requests with Poisson arrivals, meshes uniform over
    {61x21, 121x41, 181x61, 241x81} on x in [-16, 8], y in [0, 12],
    F ~ U[0.5, 1.0], eps ~ U[0.05, 0.4] (seed 0).  First a closed-loop run
    (all requests at once) measures the mixed-precision capacity; the arrival
    rate is set to 80% of it.  Then the same arrival sequence is served in
    mixed precision (FP32-Kahan inner JVPs, FP64 fallback) and in plain FP64,
    each by a warmed server (preconditioners cached per mesh and F bucket)."""
    import numpy as np
    dom = inputs.SERVING_DOMAIN

    dump = [] if out_dir else None

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
        if dump is not None:
            dump.append([{"N": q[1], "M": q[2], "F": q[3], "eps": q[4], "status": r.status,
                          "wait_s": r.t_admit_s - r.t_submit_s,
                          "service_s": r.t_done_s - r.t_admit_s, "newton": r.newton_iters,
                          "gmres": r.gmres_iters} for q, r in zip(reqs, res)])
        errs = [r.fp32_error for r in res if r.fp32_error >= 0]
        return {"requests": len(res), "converged": ok,
                "fallbacks": sum(r.used_fallback for r in res),
                "wall_s": wall, "solves_per_s": len(res) / wall,
                "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_newton": float(np.mean([r.newton_iters for r in res])),
                "mean_gmres": float(np.mean([r.gmres_iters for r in res])),
                "mean_evals": float(np.mean([r.residual_evals for r in res])),
                "max_fp32_error": float(max(errs)) if errs else None}

    base = inputs.serving_requests(nreq, 1.0, 0)
    out = {}
    servers = {}
    for prec in ("fp32", "fp64"):
        servers[prec] = api.Server(hbm_budget_bytes=64e9, max_slots=32, precision=prec,
                                   fallback_fp64=True, q_blocks=-1)
        out[f"closed_loop_{prec}"] = run(servers[prec], base)   # warms the caches
        print(f"serving closed loop {prec}: {out[f'closed_loop_{prec}']}", file=sys.stderr,
              flush=True)
    capacity = out["closed_loop_fp32"]["solves_per_s"]
    rate = fixed_rate if fixed_rate else 0.8 * capacity
    reqs = inputs.serving_requests(nreq, rate, 0)
    for prec in ("fp32", "fp64"):
        out[f"poisson_{prec}"] = run(servers[prec], reqs, rate=rate)
        servers[prec].close()
        print(f"serving poisson {prec}: {out[f'poisson_{prec}']}", file=sys.stderr, flush=True)
    out["arrival_rate_per_s"] = rate
    if dump is not None:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "serving_requests.json"), "w") as f:
            json.dump(dump, f)
    how = "fixed" if fixed_rate else "80% of closed-loop mixed capacity"
    out["workload"] = (f"serving: {nreq} requests, Poisson arrivals at {rate:.2f}/s ({how}), "
                       f"meshes 61x21/121x41/181x61/241x81 on "
                       f"[-16, 8]x[0, 12], F~U[0.5,1], eps~U[0.05,0.4], seed 0, q by mesh "
                       f"(5 for N <= 200, 8 beyond)")
    return out


def serving(args):
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()
    out = serving_runs(api, inputs, args.requests, args.serving_rate, args.out_dir)
    line = {"metric": METRIC,
            "value": out["poisson_fp32"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.requests, "warmup": args.requests, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": out["workload"]},
            "p50_latency_s": out["poisson_fp32"]["p50_latency_s"],
            "p99_latency_s": out["poisson_fp32"]["p99_latency_s"],
            "arrival_rate_per_s": out["arrival_rate_per_s"], "runs": out}
    print(json.dumps(line), flush=True)


def _line(value, unit, workload, extra, dtype="f64", higher=True):
    return {"metric": METRIC,
            "value": value, "unit": unit, "n_gpus": 1, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": {"workload": workload}, **extra}


def residuals():
    """Whole-residual throughput (prelude, pair sum and finish) on the 31x11, 181x61, 361x121
    and 721x241 workloads from a
    smooth synthetic state, each precision timed over repeated calls with HIP events."""
    import torch
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()
    rows = {}
    for name, cfg, reps in (("31x11", inputs.W31X11, 50), ("181x61", inputs.W181X61, 50),
                            ("361x121", inputs.W361X121, 10), ("721x241", inputs.W721X241, 3)):
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
    print(json.dumps(_line(rows["721x241_fp64"]["pairs_per_s"], "pairs/s",
                           "whole residual E(u) on 31x11, 181x61, 361x121 and 721x241 (smooth "
                           "state), FP64 and FP32-Kahan",
                           {"rows": rows})), flush=True)


def workloads():
    """361x121 on the paper's domain, F in {0.5, 0.7, 1.0} x eps in {0.1, 0.3},
    each solved in FP64 and in mixed precision with one preconditioner per F (q = 8).
    721x241, F = 0.7, eps continued 0.1 -> 0.5 in mixed precision (q = 16), with
    FP64 solves at the first and last eps for comparison."""
    import torch
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()
    kw = dict(inputs.LARGE_SOLVE)

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

    out = {"361x121": [], "721x241": []}
    c3 = inputs.W361X121
    for F in inputs.W361X121_F:
        P, tb = build(dict(c3, F=F), 8)
        for eps in inputs.W361X121_EPS:
            _, z64, r64 = timed(F, eps, c3, "fp64", P)
            _, z32, r32 = timed(F, eps, c3, "fp32", P)
            out["361x121"].append({"F": F, "eps": eps, "build_s": tb, "fp64": r64, "mixed": r32,
                                   "zeta_mixed_vs_fp64": (z64 - z32).abs().max().item()})
            print(f"361x121 F={F} eps={eps}: fp64 {r64['s']:.2f}s mixed {r32['s']:.2f}s",
                  file=sys.stderr, flush=True)
        P.close()
    c4 = inputs.W721X241
    P, tb = build(c4, inputs.Q_BLOCKS[(c4["N"], c4["M"])])
    out["721x241_build_s"] = tb
    u = None
    for eps in inputs.W721X241_EPS:
        um, zm, rm = timed(c4["F"], eps, c4, "fp32", P, u)
        rec = {"eps": eps, "mixed": rm}
        if eps in (inputs.W721X241_EPS[0], inputs.W721X241_EPS[-1]):
            _, z64, r64 = timed(c4["F"], eps, c4, "fp64", P, u)
            rec["fp64"] = r64
            rec["zeta_mixed_vs_fp64"] = (z64 - zm).abs().max().item()
        out["721x241"].append(rec)
        print(f"721x241 eps={eps}: mixed {rm['s']:.2f}s status {rm['status']}", file=sys.stderr,
              flush=True)
        if rm["status"] != 0:
            break
        u = um
    P.close()
    n = len(out["721x241"])
    total = sum(r["mixed"]["s"] for r in out["721x241"])
    print(json.dumps(_line(n / total, "solves/s",
                           "721x241 eps continuation 0.1..0.5 (mixed, q=16); "
                           "361x121 F x eps grid in FP64 and mixed (q=8)",
                           {"runs": out}, dtype="f32+f64")), flush=True)


# Function-evaluation times of the paper's Table 1 (seconds; eps = 1, F = 0.7):
# multicore MATLAB on the desktop, on the workstation, and MATLAB with the M2090 GPU.
PAPER_TABLE1_S = {(91, 31): (1.43, 0.87, 0.02), (181, 61): (11.26, 4.38, 0.18),
                  (271, 91): (54.47, 20.40, 0.83), (361, 121): (169.46, 64.35, 2.52),
                  (451, 151): (410.34, 153.91, 6.04)}


def _continue(api, cfg, F, eps_list, prec, q, kw, log):
    """eps continuation with one preconditioner: each root starts the next solve."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = api.Preconditioner(api.Problem(**dict(cfg, F=F, eps=eps_list[0])), q)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    u, z, steps = None, None, []
    for eps in eps_list:
        t0 = time.perf_counter()
        un, zn, info = api.solve(F, eps, cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"],
                                 precision=prec, precond=P, u0=u, **kw)
        torch.cuda.synchronize()
        rec = {"eps": eps, "status": info.status, "newton": info.newton_iters,
               "gmres": info.gmres_iters, "evals": info.residual_evals,
               "backtracks": info.linesearch_backtracks, "final_norm": info.final_norm,
               "s": time.perf_counter() - t0, "zeta_max": zn.max().item(),
               "zeta_min": zn.min().item()}
        steps.append(rec)
        log(f"  {cfg['N']}x{cfg['M']} F={F} eps={eps:.2f} {prec}: {rec}")
        if info.status != 0:
            break
        u, z = un, zn
    P.close()
    return u, z, {"build_s": build_s, "q": q, "precision": prec, "steps": steps}


def table1(out_dir=None):
    """The paper's headline workload, eps = 1 and F = 0.7 (results section):
    function-evaluation times on the Table-1 meshes beside Table 1; roots at eps = 1
    on 91 x 31, 361 x 121 and 721 x 241 by eps continuation in steps of 0.1 from the
    flat surface; their centrelines zeta(x, 0); and F = 1.4 on 721 x 241 with spacing
    0.3 from x_1 = -56.  Writes the centrelines to table1_centrelines.json in out_dir
    when that folder exists."""
    import numpy as np
    import torch
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()

    def log(m):
        print(m, file=sys.stderr, flush=True)

    out = {"evaluations": {}, "continuation": {}, "centreline": {}}
    for (N, M), dom in inputs.TABLE1.items():
        cfg = dict(N=N, M=M, F=0.7, eps=1.0, **dom)
        row = {"domain": dom, "spacing": (dom["xN"] - dom["x1"]) / (N - 1)}
        for prec in ("fp64", "fp32"):
            p = api.Problem(**cfg, precision=prec)
            u = torch.tensor(inputs.smooth_state(N, M, 0.05, 3), device="cuda")
            E = api.residual(p, u)
            torch.cuda.synchronize()
            reps = max(3, min(200, int(2e10 / p.pairs)))
            s = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(reps):
                api.residual(p, u, out=E)
            e.record()
            torch.cuda.synchronize()
            ms = s.elapsed_time(e) / reps
            row[f"{prec}_ms"] = ms
            row[f"{prec}_pairs_per_s"] = p.pairs / (ms * 1e-3)
        paper = PAPER_TABLE1_S[(N, M)]
        row["paper_s"] = {"matlab_desktop": paper[0], "matlab_workstation": paper[1],
                          "matlab_m2090_gpu": paper[2]}
        row["speedup_fp64_vs_paper_gpu"] = paper[2] / (row["fp64_ms"] * 1e-3)
        out["evaluations"][f"{N}x{M}"] = row
        log(f"E(u) {N}x{M}: fp64 {row['fp64_ms']:.3f} ms fp32 {row['fp32_ms']:.3f} ms "
            f"(paper GPU {paper[2]} s)")
    kw = dict(inputs.LARGE_SOLVE)
    eps_list = [round(0.1 * k, 1) for k in range(1, 11)]
    runs = [("91x31", dict(N=91, M=31, **inputs.TABLE1[(91, 31)]), 0.7, "fp64", 30),
            ("361x121", dict(inputs.W361X121), 0.7, "fp64", 8),
            ("721x241", dict(inputs.W721X241), 0.7, "fp32", 16),
            ("721x241_F1.4", dict(inputs.W721X241_F14), 1.4, "fp32", 16)]
    for name, cfg, F, prec, q in runs:
        cfg = dict(cfg)
        cfg.pop("eps", None)
        cfg["F"] = F
        t0 = time.perf_counter()
        u, z, rec = _continue(api, cfg, F, eps_list, prec, min(q, cfg["M"] - 1), kw, log)
        rec["total_s"] = time.perf_counter() - t0
        out["continuation"][name] = rec
        if z is not None and rec["steps"][-1]["status"] == 0:
            zz = z.cpu().numpy().reshape(cfg["M"], cfg["N"])
            x = cfg["x1"] + np.arange(cfg["N"]) * (cfg["xN"] - cfg["x1"]) / (cfg["N"] - 1)
            out["centreline"][name] = {"x": x.tolist(), "zeta": zz[0].tolist()}
    cl = out["centreline"]
    cmp = {}
    if "361x121" in cl and "721x241" in cl:
        a = np.array(cl["361x121"]["zeta"])
        b = np.array(cl["721x241"]["zeta"])[::2]   # same x_1, half the spacing
        x = np.array(cl["361x121"]["x"])
        near = x <= 15.0
        cmp["361_vs_721_max_abs"] = float(np.abs(a - b).max())
        cmp["361_vs_721_max_abs_x_le_15"] = float(np.abs(a - b)[near].max())
    if "91x31" in cl and "721x241" in cl:
        xa = np.array(cl["91x31"]["x"])
        za = np.array(cl["91x31"]["zeta"])
        zb = np.interp(xa, np.array(cl["721x241"]["x"]), np.array(cl["721x241"]["zeta"]))
        cmp["91_vs_721_max_abs"] = float(np.abs(za - zb).max())
    for name, c in cl.items():
        zc = np.array(c["zeta"])
        xc = np.array(c["x"])
        cmp[f"{name}_zeta_max_at_x"] = [float(zc.max()), float(xc[zc.argmax()])]
        cmp[f"{name}_zeta_min_at_x"] = [float(zc.min()), float(xc[zc.argmin()])]
    out["centreline_comparison"] = cmp
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "table1_centrelines.json"), "w") as f:
            json.dump(out["centreline"], f)
    del out["centreline"]
    ev = out["evaluations"]
    print(json.dumps(_line(ev["361x121"]["fp64_pairs_per_s"], "pairs/s",
                           "the paper's eps = 1, F = 0.7 workload: E(u) on the Table-1 meshes, "
                           "continuation to eps = 1 (91x31, 361x121, 721x241; F = 1.4 on 721x241 "
                           "with spacing 0.3 from x_1 = -56)", {"runs": out}, dtype="f64")),
          flush=True)


def precond_study(out_dir=None):
    """The preconditioner study (preconditioning section): GMRES iterations per
    Newton step against the block bandwidth b = 2q + 1 at 361 x 121 (eps = 1, F = 0.7,
    from the eps = 0.9 root) and for cold solves of the benched 721 x 241 workload, and
    the spectra of J and J P^-1 on 45 x 13 (spacing 0.4,
    x_1 = -9, eps = 1, F = 0.7, at the flat state) with J assembled from GPU JVP
    columns and P^-1 from preconditioner applies of the unit vectors."""
    import numpy as np
    import torch
    from paper_1403_5044_amd import api, inputs
    from paper_1403_5044_amd import _lib
    _lib.load()

    def log(m):
        print(m, file=sys.stderr, flush=True)

    out = {"bandwidth_sweep": [], "spectra": {}}
    cfg = dict(inputs.W361X121)
    cfg.pop("eps")
    kw = dict(inputs.LARGE_SOLVE)
    u09, _, rec = _continue(api, cfg, 0.7, [round(0.1 * k, 1) for k in range(1, 10)], "fp64",
                            8, kw, log)
    out["start"] = {"eps": 0.9, "continuation": rec}
    for q in range(0, 16):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = api.Preconditioner(api.Problem(**cfg, eps=1.0), q)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, _, info = api.solve(0.7, 1.0, cfg["N"], cfg["M"], cfg["x1"], cfg["xN"], cfg["yM"],
                               precond=P, u0=u09, **kw)
        torch.cuda.synchronize()
        r = {"b": 2 * q + 1, "q": q, "status": info.status, "newton": info.newton_iters,
             "gmres": info.gmres_iters, "evals": info.residual_evals,
             "gmres_per_newton": info.gmres_iters / max(1, info.newton_iters),
             "build_s": tb, "solve_s": time.perf_counter() - t0}
        P.close()
        out["bandwidth_sweep"].append(r)
        log(f"b={2 * q + 1}: {r}")
    # the same sweep on the finest mesh (spacing 0.075, half that of 361 x 121): cold FP64
    # solves of the benched workload (eps = 0.1 from the flat surface), set-up included
    c4 = dict(inputs.W721X241)
    out["bandwidth_sweep_721x241"] = []
    for q in (8, 12, 14, 16, 18, 20, 24):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = api.solve(c4["F"], c4["eps"], c4["N"], c4["M"], c4["x1"], c4["xN"],
                               c4["yM"], q_blocks=q, **kw)
        torch.cuda.synchronize()
        r = {"b": 2 * q + 1, "q": q, "status": info.status, "newton": info.newton_iters,
             "gmres": info.gmres_iters, "evals": info.residual_evals,
             "gmres_per_newton": info.gmres_iters / max(1, info.newton_iters),
             "build_s": info.time_precond_s, "solve_s": time.perf_counter() - t0,
             "band_factor_bytes": c4["M"] * (2 * q + 1) * c4["N"] ** 2 * 8}
        out["bandwidth_sweep_721x241"].append(r)
        log(f"721x241 b={2 * q + 1}: {r}")
    # spectra on 45 x 13
    N, M = 45, 13
    c = dict(N=N, M=M, x1=-9.0, xN=-9.0 + 0.4 * (N - 1), yM=0.4 * (M - 1), F=0.7, eps=1.0)
    p = api.Problem(**c)
    n = p.n_unknowns
    u0 = torch.tensor(inputs.flat_state(N, M), device="cuda")
    Eu = api.residual(p, u0)
    Jt = torch.empty(n, n, dtype=torch.float64, device="cuda")   # row i = column i of J
    ecol = torch.zeros(n, dtype=torch.float64, device="cuda")
    for i in range(n):
        ecol.zero_()
        ecol[i] = 1.0
        api.jvp(p, u0, Eu, ecol, out=Jt[i])
    Jh = Jt.cpu().numpy().T
    ev = np.linalg.eigvals(Jh)
    out["spectra"]["J"] = _spectrum_summary(ev)
    spectra = {"J": [ev.real.tolist(), ev.imag.tolist()]}
    for q in (0, 1, 2, M - 1):
        P = api.Preconditioner(p, q)
        Pt = torch.empty(n, n, dtype=torch.float64, device="cuda")   # row i = P^-1 e_i
        for i in range(n):
            ecol.zero_()
            ecol[i] = 1.0
            P.apply(ecol, out=Pt[i])
        torch.cuda.synchronize()
        P.close()
        evp = np.linalg.eigvals(Jh @ Pt.cpu().numpy().T)
        key = f"JPinv_b{2 * q + 1}" if q < M - 1 else "JPinv_full"
        out["spectra"][key] = _spectrum_summary(evp)
        spectra[key] = [evp.real.tolist(), evp.imag.tolist()]
        log(f"{key}: {out['spectra'][key]}")
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "precond_spectra.json"), "w") as f:
            json.dump(spectra, f)
    best = min(out["bandwidth_sweep"], key=lambda r: r["build_s"] + r["solve_s"])
    print(json.dumps(_line(best["gmres_per_newton"], "GMRES iterations per Newton step",
                           "preconditioner study: block bandwidth sweep at 361x121 (eps = 1, "
                           "F = 0.7, from the eps = 0.9 root); spectra of J and J P^-1 on 45x13",
                           {"runs": out}, higher=False)), flush=True)


def _spectrum_summary(ev):
    import numpy as np
    d = np.abs(ev - 1.0)
    return {"n": int(ev.size), "re_min": float(ev.real.min()), "re_max": float(ev.real.max()),
            "abs_im_max": float(np.abs(ev.imag).max()), "abs_min": float(np.abs(ev).min()),
            "abs_max": float(np.abs(ev).max()), "max_dist_from_1": float(d.max()),
            "frac_within_0.1_of_1": float((d <= 0.1).mean()),
            "frac_within_0.5_of_1": float((d <= 0.5).mean())}


if __name__ == "__main__":
    main()
