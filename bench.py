#!/usr/bin/env python3
"""Benchmark of the FAS multigrid Monge-Ampere solver on one MI355X.

Default workload: the served stream -- Poisson arrivals of solve requests
with grid sizes 65^3 / 129^3 / 257^3 / 385^3 (p = .4/.3/.2/.1), quadratic or
exp-cos data, relative discrete L2 residual 1e-8, through the
continuous-batching server (HBM-budgeted admission, resident hierarchies, one
resident batch per size class).  One step is 16 requests of the arrival
trace; the arrival rate is 0.8 x the measured capacity of the same mix
solved one request at a time.  The request data are on the device before
the clock starts.  The same trace is served in the plain FP64 form (the
value), in the mixed FP32/FP64 form and with a 4 GiB budget that forces
admission queueing.  Other workloads:
  quadratic129, example4_17, expcos257, expcos385   single solves (one step =
            one solve, Poisson initial guess, FAS V(2,2) to 1e-8);
  batch64   64 seeded solves (sizes 33^3..129^3, quadratic or exp-cos) run
            as one batch; one step = the whole batch;
  *_fmg, gs_*, ex2d*  the Section 4 protocol, the standalone Gauss-Seidel
            solver and the 2D variant.
Before timing a single solve or the batch, the autotuner picks the engine's
launch shapes on the same solvers and data (outside the timed region;
--no-tune keeps the defaults).

Prints one JSON line: solves/s (value), p50/p99 latency, grid-point
updates/s, the finest-level smoother's algorithmic bandwidth against the HBM
peak (HIP events on the engine stream around its launches, in an
instrumented pass), and the CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Counter-measured bytes per launch of the dominant kernel (FETCH_SIZE and
# WRITE_SIZE, each scaled by the same counter's reading for a plain copy of
# known size), keyed by (workload, kernel); valid only for the kernel as it
# was profiled.
TRAFFIC = {("served", "k_zsweep"): 1.785e9}   # profiles/k_zsweep_expcos385.md
METRIC = "solves/s + p50/p99 latency at 1e-8 rel residual; smoother GB/s vs HBM peak"
SINGLE = {
    # name: (kind, n, seed, tol, start)
    "quadratic129": ("quadratic", 128, 1001, 1e-8, "poisson"),
    "example4_17": ("example4", 16, 0, 1e-10, "poisson"),
    "expcos257": ("exp_cos", 256, 3001, 1e-8, "poisson"),
    "expcos385": ("exp_cos", 384, 5001, 1e-8, "poisson"),
    # Section 4 protocol (FMG-FAS start, tolerance 1e-6) on Examples 4-7
    "example4_129_fmg": ("example4", 128, 0, 1e-6, "fmg"),
    "example5_129_fmg": ("example5", 128, 0, 1e-6, "fmg"),
    "example6_129_fmg": ("example6", 128, 0, 1e-6, "fmg"),
    "example7_129_fmg": ("example7", 128, 0, 1e-6, "fmg"),
}
# the standalone Gauss-Seidel solver from 1.01 u to 1e-6 (Table 3 protocol)
GS = {"gs_example4_33": ("example4", 32, 1e-6)}
# 2D variant, Section 4 protocol (FMG start, tolerance 1e-6), red-black
TWO_D = {"ex2d1_8193_fmg": (1, 8192), "ex2d2_8193_fmg": (2, 8192), "ex2d3_8193_fmg": (3, 8192),
         "ex2d1_1025_fmg": (1, 1024)}
WORKLOADS = sorted(SINGLE) + sorted(GS) + sorted(TWO_D) + ["batch64", "served"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (served: blocks of 16 requests); default per workload")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="served", choices=WORKLOADS)
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: fp64, except batch64 (mixed)")
    ap.add_argument("--init", default=None, choices=["poisson", "fmg"],
                    help="single solves: Poisson initial guess or the Section 4 protocol "
                         "(one FMG-FAS iteration as the first cycle); default per workload")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tuned", default=None,
                    help="coarse_n,max_blocks[,strip_rows[,block_n]] to use instead of running the "
                         "autotuner")
    ap.add_argument("--copy-calibration", type=float, default=None, metavar="MB",
                    help="only run 20 plain device copies of MB megabytes (counter "
                         "calibration for the traffic figures) and exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only run the instrumented 385^3 solves behind the served line's "
                         "roofline and print that record (for kernel traces and counters)")
    ap.add_argument("--rate", type=float, default=None,
                    help="served: arrivals per second (default 0.8 x the measured "
                         "one-at-a-time capacity of the size mix)")
    ap.add_argument("--budget-gb", type=float, default=None, help="served: HBM budget")
    ap.add_argument("--lanes", default="65/129/257/385",
                    help="served: size classes in points per side, '/' between classes and "
                         "',' inside one (one resident batch, ticking on its own stream, per "
                         "class); 'none' for a single batch")
    return ap.parse_args()


def roofline(reps, traffic=None):
    sec = sum(r["smooth_seconds"] for r in reps)
    by = sum(r["smooth_bytes"] for r in reps)
    la = sum(r["smooth_launches"] for r in reps)
    ach = by / sec / 1e9 if sec > 0 else 0.0
    out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
           "kernel": ("finest-level smoother launches: z-stream sweeps (k_zsweep) on levels at "
                      "or above the z-stream threshold, else colour phases (k_batched) or block "
                      "sweeps (k_bsweep); 24 B per interior node per sweep, plus 16 B per "
                      "coarse node for z-stream sweeps that also prolong"),
           "avg_launch_us": 1e6 * sec / max(la, 1), "launches": la,
           "alg_bytes_per_launch": by / max(la, 1)}
    if traffic is not None:
        out["traffic_unit"] = "bytes per launch (counters)"
    if la == 0:
        # a grid of n <= coarse_n has no row-kernel sweep: all its levels run
        # in one single-workgroup launch per cycle, bound by the dependent
        # FP64 chain of each phase rather than by memory
        out.update({"bound": "latency", "achieved": None, "frac": None,
                    "kernel": "none: every level runs in k_tail_lds (one workgroup per "
                              "solve, latency bound)"})
    return out


def cpu_baseline(kind, n, seed, tol, init="poisson"):
    """The oracle (serial C, one core) on a bounded sample of the workload:
    the full solve when it fits in ~30 s, else V-cycles on it for ~20 s."""
    import oracle
    from paper_1411_7018_amd import problems as P

    p = P.make(kind, n, seed)
    u = P.initial_guess(p)
    if n <= 128:
        t0 = time.perf_counter()
        st, rep, _ = oracle.solve(u, p.f, oracle.params(tol=tol, init=init))
        dt = time.perf_counter() - t0
        start = (f"{rep.init_cycles} Poisson + " if init == "poisson" else "FMG-FAS + ")
        return {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": f"one full solve of the same {n + 1}^3 problem "
                          f"({start}{rep.cycles} cycles in all, {dt:.1f} s)"}
    oracle.poisson_init(u, p.f, oracle.params())
    t0 = time.perf_counter()
    cyc = 0
    while time.perf_counter() - t0 < 20.0:
        oracle.vcycle(u, p.f, oracle.params())
        cyc += 1
    dt = (time.perf_counter() - t0) / cyc
    return {"value": dt, "unit": "s per V-cycle", "cores": 1, "kind": "oracle",
            "sample": f"{cyc} FAS V(2,2) cycles on the same {n + 1}^3 problem"}


def base_line(args, value, steps, warmup, elapsed, lat, precision):
    return {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": 1e3 * elapsed / max(steps, 1),
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64", "data": "synthetic",
    }


def pick_tuning(args, solvers, us, fs, ticks):
    from paper_1411_7018_amd import autotune

    if args.tuned:
        vals = [int(v) for v in args.tuned.split(",")]
        cn, mb, sr, bn = (vals + [0, 0])[:4]
        for s in solvers:
            s.retune(coarse_n=cn, max_blocks=mb, strip_rows=sr, block_n=bn)
        return autotune.Choice(cn, mb, sr, bn, float("nan"), [])
    if args.no_tune:
        return None
    return autotune.tune(solvers, us, fs, ticks=ticks)


def copy_calibration(mb):
    """Plain device-to-device copies of a known size: the reference against
    which the FETCH_SIZE / WRITE_SIZE counters of the solver kernels are
    scaled."""
    import torch

    count = int(mb * 1e6) // 8
    a = torch.ones(count, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": count * 8, "copies": 20}), flush=True)


def diff_vs_fp64(ns, us_init, fs, us_done, tol, init="poisson"):
    """Max-norm difference of mixed-precision results from the same problems
    solved by the FP64 path (outside the timed region): the agreement the
    mixed form reaches at the benchmark's stopping tolerance."""
    import torch

    from paper_1411_7018_amd import Solver

    worst = 0.0
    for n, u0, f, u in zip(ns, us_init, fs, us_done):
        s = Solver(n, precision="fp64")
        w = u0.clone()
        s.solve(w, f, tol=tol, init=init)
        torch.cuda.synchronize()
        worst = max(worst, float((w - u).abs().max()))
        s.close()
        del w
    return worst


def retune_like(solvers, choice):
    """Give the instrumented solvers the launch shape the timed ones use."""
    if choice is not None:
        for s in solvers:
            s.retune(coarse_n=choice.coarse_n, max_blocks=choice.max_blocks,
                     strip_rows=choice.strip_rows, block_n=choice.block_n,
                     tile_config=choice.tile_config, zsweep_n=choice.zsweep_n)


def instrumented(reps, elapsed, per_step):
    """Where the roofline's launch durations come from."""
    return {"pass": "second pass over the same steps, HIP events on the engine stream "
                    "around every group of finest-level sweep launches (one graph per "
                    "segment between them)",
            "solves_per_s": per_step * len(reps) / elapsed}


def tune_note(choice):
    if choice is None:
        return None
    return {"coarse_n": choice.coarse_n, "max_blocks": choice.max_blocks,
            "strip_rows": choice.strip_rows, "block_n": choice.block_n,
            "tile_config": choice.tile_config, "zsweep_n": choice.zsweep_n,
            "ms_per_tick": 1e3 * choice.seconds_per_tick}


def run_single(args, precision):
    import torch

    from paper_1411_7018_amd import Solver, problems as P

    kind, n, seed, tol, start = SINGLE[args.workload]
    init = args.init or start
    steps = args.steps or 20
    warmup = 3 if args.warmup is None else args.warmup
    prob = P.make(kind, n, seed)
    dev = torch.device("cuda:0")
    u_init = torch.from_numpy(P.initial_guess(prob)).to(dev)
    f = torch.from_numpy(prob.f).to(dev)
    u = torch.empty_like(u_init)
    # The timed solver replays one graph per cycle.  A second, instrumented
    # solver with the same launch shape splits each cycle's graph at the
    # finest-level sweep boundaries to time those launches with HIP events;
    # its pass runs after the timed one and feeds only the roofline.
    s = Solver(n, precision=precision)
    sp = Solver(n, precision=precision, profile=1)
    choice = pick_tuning(args, [s], [u_init], [f], ticks=4)
    retune_like([sp], choice)

    def step(solver=s):
        u.copy_(u_init)
        return solver.solve(u, f, tol=tol, init=init)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, reps = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        reps.append(step())
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last = reps[-1]
    err = float(np.abs(u.cpu().numpy() - prob.u_exact).max())
    dmix = (diff_vs_fp64([n], [u_init], [f], [u], tol, init) if precision == "mixed" else None)
    step(sp)
    torch.cuda.synchronize()
    preps = []
    tp = time.perf_counter()
    for _ in range(steps):
        preps.append(step(sp))
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    out = base_line(args, steps / elapsed, steps, warmup, elapsed, lat, precision)
    out["config"] = {
        "workload": f"{kind} {n + 1}^3 single solve, seed {seed}, tol {tol:g}, "
                    + ("Poisson initial guess" if init == "poisson" else
                       "FMG-FAS start (r0 of the zero-interior start)")
                    + f", FAS V(2,2), 4-colour nonlinear GS, {precision}",
        "n": n, "tol": tol, "precision": precision, "init": init,
        "tuned": tune_note(choice)}
    out.update({"updates_per_s": sum(r["point_updates"] for r in reps) / elapsed,
                "cycles": last["cycles"], "init_cycles": last["init_cycles"],
                "rel_res": last["rel_res"], "max_err_vs_exact": err,
                **({"max_abs_diff_vs_fp64": dmix} if dmix is not None else {}),
                "roofline": dict(roofline(preps, TRAFFIC.get((args.workload, precision))),
                                 **instrumented(preps, tp, 1))})
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(kind, n, seed, tol, init)
    return out


def run_gs(args, precision):
    import torch

    from paper_1411_7018_amd import Solver, problems as P

    kind, n, tol = GS[args.workload]
    steps = args.steps or 5
    warmup = 1 if args.warmup is None else args.warmup
    prob = P.make(kind, n)
    u0 = torch.from_numpy(P.initial_guess(prob, 1.01 * prob.u_exact)).cuda()
    f = torch.from_numpy(prob.f).cuda()
    u = torch.empty_like(u0)
    s = Solver(n, precision=precision)

    def step():
        u.copy_(u0)
        return s.gs_solve(u, f, tol=tol)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, reps = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        reps.append(step())
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = base_line(args, steps / elapsed, steps, warmup, elapsed, lat, "fp64")
    out["config"] = {"workload": f"standalone nonlinear Gauss-Seidel (4-colour) on {kind} "
                                 f"{n + 1}^3 from 1.01 u to relative residual {tol:g}",
                     "n": n, "tol": tol}
    out.update({"sweeps": reps[-1]["cycles"], "rel_res": reps[-1]["rel_res"],
                "max_err_vs_exact": float(np.abs(u.cpu().numpy() - prob.u_exact).max()),
                "updates_per_s": sum(r["point_updates"] for r in reps) / elapsed})
    return out


def run_2d(args, precision):
    import torch

    from paper_1411_7018_amd import problems as P
    from paper_1411_7018_amd.solver2d import Solver2D

    ex, n = TWO_D[args.workload]
    steps = args.steps or 5
    warmup = 1 if args.warmup is None else args.warmup
    prob = P.example2d(ex, n)
    u0 = torch.from_numpy(P.initial_guess2(prob)).cuda()
    f = torch.from_numpy(prob.f).cuda()
    u = torch.empty_like(u0)
    s = Solver2D(n)

    def step():
        u.copy_(u0)
        return s.solve(u, f, tol=1e-6)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, reps = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        reps.append(step())
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = base_line(args, steps / elapsed, steps, warmup, elapsed, lat, "fp64")
    out["config"] = {"workload": f"2D Example {ex} on {n + 1}^2, FMG-FAS start, tolerance 1e-6, "
                                 f"red-black ordering, half-weighting, V(2,2)",
                     "n": n, "example": ex}
    out.update({"cycles": reps[-1]["cycles"], "rel_res": reps[-1]["rel_res"],
                "max_err_vs_exact": float(np.abs(u.cpu().numpy() - prob.u_exact).max()),
                "updates_per_s": sum(r["point_updates"] for r in reps) / elapsed})
    return out


def run_batch(args, precision):
    import torch

    from paper_1411_7018_amd import Solver, problems as P
    from paper_1411_7018_amd.batch import solve_batch

    steps = args.steps or 5
    warmup = 1 if args.warmup is None else args.warmup
    specs = P.batch_specs(64)
    data = [P.make_device(k, n, sd) for k, n, sd in specs]
    us0 = [d[0] for d in data]
    fs = [d[1] for d in data]
    us = [torch.empty_like(u) for u in us0]
    solvers = [Solver(n, precision=precision) for _, n, _ in specs]
    psolvers = [Solver(n, precision=precision, profile=1) for _, n, _ in specs]
    choice = pick_tuning(args, solvers, us0, fs, ticks=3)
    retune_like(psolvers, choice)

    def step(group=solvers):
        for u, u0 in zip(us, us0):
            u.copy_(u0)
        st, reps = solve_batch(group, us, fs, tol=1e-8)
        if st != 0:
            raise RuntimeError(f"batch status {st}")
        return reps

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, allreps = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        allreps.append(step())
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nsol = len(specs)
    dmix = (diff_vs_fp64([n for _, n, _ in specs], us0, fs, us, 1e-8)
            if precision == "mixed" else None)
    step(psolvers)
    torch.cuda.synchronize()
    preps = []
    tp = time.perf_counter()
    for _ in range(steps):
        preps.append(step(psolvers))
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    out = base_line(args, steps * nsol / elapsed, steps, warmup, elapsed, lat, precision)
    pts = sum((n + 1) ** 3 for _, n, _ in specs)
    out["config"] = {
        "workload": f"batch of {nsol} seeded solves (sizes 33^3..129^3, quadratic or "
                    f"exp-cos, {pts / 1e6:.1f}M grid points), tol 1e-8, Poisson initial "
                    f"guess, FAS V(2,2), {precision}, one launch per level phase",
        "solves": nsol, "tol": 1e-8, "precision": precision, "tuned": tune_note(choice),
        "latency": "per batch step"}
    # smooth_* of a batch report are the whole batch's totals: use one per step
    out.update({"updates_per_s": sum(r["point_updates"] for reps in allreps for r in reps)
                / elapsed,
                "max_cycles": max(r["cycles"] for r in allreps[-1]),
                "max_rel_res": max(r["rel_res"] for r in allreps[-1]),
                **({"max_abs_diff_vs_fp64": dmix} if dmix is not None else {}),
                "roofline": dict(roofline([reps[0] for reps in preps]),
                                 **instrumented(preps, tp, nsol))})
    return out


STEP_REQUESTS = 16       # served stream: requests of the arrival trace per bench step
SMALL_BUDGET_GB = 4.0    # served stream: the budget that forces admission queueing


def solo_capacity(precision):
    """Solves/s of the served size mix when every request is solved alone,
    one after the other: 1 / sum_n w_n t_n with t_n the solo solve time of an
    n grid (mean of a quadratic and an exp-cos problem, graphs warm)."""
    import torch

    from paper_1411_7018_amd import Solver, problems as P

    times = {}
    for n in P.SERVE_SIZES:
        ts = []
        s = Solver(n, precision=precision)
        for kind, seed in (("quadratic", 91), ("exp_cos", 92)):
            u0, f = P.make_device(kind, n, seed)
            u = u0.clone()
            s.solve(u, f, tol=1e-8)
            u.copy_(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve(u, f, tol=1e-8)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            del u0, f, u
        s.close()
        times[n] = sum(ts) / len(ts)
    mean = sum(w * times[n] for n, w in zip(P.SERVE_SIZES, P.SERVE_WEIGHTS))
    return 1.0 / mean, times


def serve(server, trace, keep=None):
    """Serve one arrival trace whose request data are already on the device
    (the client's payloads, made before the clock starts)."""
    import torch

    from paper_1411_7018_amd import problems as P
    from paper_1411_7018_amd.server import requests_from_trace

    reqs = requests_from_trace(trace)
    for r in reqs:
        r.payload = P.make_device(r.kind, r.n, r.seed)
    torch.cuda.synchronize()
    server.keep_results = keep is not None
    st = server.run(reqs)
    torch.cuda.synchronize()
    if keep is not None:
        for r in reqs:
            if r.rid not in keep:
                r.u = None
    return st, reqs


def served_cpu_baseline(cycles_by_n):
    """The oracle (serial C, one core) on a bounded sample of the served
    mix: one linear and one FAS V-cycle (and a residual) timed at 65^3,
    129^3 and 257^3, the 385^3 times extrapolated from 257^3 by the ratio of
    interior nodes; combined with the cycle counts the served solves took
    into seconds per request, and requests/s for the size mix."""
    import platform

    import torch

    import oracle
    from paper_1411_7018_amd import problems as P

    per, unit = {}, {}
    spent = 0.0
    timed = [n for n in P.SERVE_SIZES if n <= 256]
    for n in timed:
        u0, f = P.make_device("exp_cos", n, 777)
        u, fh = u0.cpu().numpy(), f.cpu().numpy()
        del u0, f
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        oracle.poisson_vcycle(u, oracle.poisson_rhs(fh))
        t_lin = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.vcycle(u, fh)
        t_fas = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.residual(u, fh, out=False)
        t_res = time.perf_counter() - t0
        spent += t_lin + t_fas + t_res
        unit[n] = (t_lin, t_fas, t_res)
    for n in P.SERVE_SIZES:
        if n not in unit:
            ref = max(timed)
            k = ((n - 1) / (ref - 1)) ** 3
            unit[n] = tuple(k * t for t in unit[ref])
        t_lin, t_fas, t_res = unit[n]
        init_c, main_c = cycles_by_n.get(n, (6.0, 12.0))
        per[n] = init_c * (t_lin + t_res) + main_c * (t_fas + t_res)
    mean = sum(w * per[n] for n, w in zip(P.SERVE_SIZES, P.SERVE_WEIGHTS))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        model = platform.processor() or "unknown"
    return {"value": 1.0 / mean, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_nproc": os.cpu_count(),
            "seconds_per_request": {str(n + 1): per[n] for n in P.SERVE_SIZES},
            "sample": f"one linear and one FAS V(2,2) cycle plus a residual of an exp-cos "
                      f"problem at 65^3, 129^3 and 257^3 ({spent:.1f} s in all; 385^3 "
                      f"extrapolated from 257^3 by the ratio of interior nodes), scaled by "
                      f"the mean cycle counts of the served solves of each size and averaged "
                      f"over the size mix (.4/.3/.2/.1)"}


def served_roofline():
    """Instrumented solves of a 385^3 request (the largest share of the
    served GPU time) with the served launch shape: HIP events on the engine
    stream around the finest-level smoother launches."""
    import torch

    from paper_1411_7018_amd import Solver, problems as P

    n = 384
    u0, f = P.make_device("exp_cos", n, 5001)
    sp = Solver(n, profile=1)
    u = u0.clone()
    sp.solve(u, f, tol=1e-8)
    reps = []
    t0 = time.perf_counter()
    for _ in range(2):
        u.copy_(u0)
        reps.append(sp.solve(u, f, tol=1e-8))
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    r = roofline(reps, TRAFFIC.get(("served", "k_zsweep")))
    r["kernel"] = ("finest-level smoother of a 385^3 request: z-stream sweeps (k_zsweep, all "
                   "four colour phases per launch; Monge-Ampere and Poisson sweeps; the first "
                   "post-smoothing sweep of a cycle also applies the coarse-grid correction), "
                   "24 B per interior node per sweep plus 16 B per coarse node for the "
                   "prolonging sweeps")
    r.update(instrumented(reps, tp, 1))
    r["pass"] = ("two instrumented 385^3 exp-cos solves after the served runs, HIP events on "
                 "the engine stream around every group of finest-level sweep launches")
    sp.close()
    return r


def run_served(args, precision):
    import numpy as np
    import torch

    from paper_1411_7018_amd import problems as P
    from paper_1411_7018_amd.server import GpuBackend, Server

    steps = args.steps or 16
    warmup = 2 if args.warmup is None else args.warmup
    count = steps * STEP_REQUESTS
    lanes = None
    if args.lanes and args.lanes != "none":
        # classes of grid sizes in points per side (65, 129, ...); requests carry n
        lanes = [[int(p) - 1 for p in c.split(",")] for c in args.lanes.split("/")]
    cap, solo = solo_capacity("fp64")
    rate = args.rate if args.rate is not None else 0.8 * cap
    trace = P.arrival_trace(count, rate, seed=5000)
    warm = P.arrival_trace(max(warmup * STEP_REQUESTS, 1), rate, seed=4999) if warmup else None
    budget = (int(args.budget_gb * (1 << 30)) if args.budget_gb
              else GpuBackend.budget_default())
    sample = set(range(0, count, 8))

    def form(prec, bud, keep=None, arrivals=trace):
        srv = Server(GpuBackend(precision=prec, tol=1e-8, max_slots=64), bud, max_slots=64,
                     lanes=lanes)
        if warm:
            serve(srv, warm)
        st, reqs = serve(srv, arrivals, keep)
        lat = [r.latency for r in reqs if r.status == 0]
        rec = {"solves_per_s": st.solves_per_s, "p50_ms": 1e3 * st.p50,
               "p99_ms": 1e3 * st.p99, "completed": st.completed, "rejected": st.rejected,
               "makespan_s": st.makespan, "queued": st.queued, "max_live": st.max_live,
               "peak_bytes": st.peak_bytes, "budget_bytes": bud,
               # requests that ended without meeting the tolerance: their
               # start was so close that tol x r0 lies under the FP64 floor,
               # where the residual stalls (status 4 after a few cycles)
               "not_converged": [{"n": r.n, "kind": r.kind, "seed": r.seed,
                                  "rel_res": r.report["rel_res"] if r.report else None,
                                  "cycles": r.report["cycles"] if r.report else None}
                                 for r in reqs if r.status not in (0, None) and r.status != 2]}
        reports = [(r.n, r.report) for r in reqs if r.status == 0 and r.report]
        return rec, reqs, lat, reports

    plain, preqs, plat, plain_reports = form("fp64", budget, sample)
    mixed, mreqs, _, _ = form("mixed", budget, sample)
    diffs = [float((m.u - p.u).abs().max()) for p, m in zip(preqs, mreqs)
             if p.u is not None and m.u is not None]
    mixed["max_abs_diff_vs_fp64"] = max(diffs) if diffs else None
    mixed["diff_sample"] = f"{len(diffs)} requests (every 8th), max-norm against the FP64 result"
    del preqs, mreqs
    small, sreqs, _, _ = form("fp64", int(SMALL_BUDGET_GB * (1 << 30)))
    del sreqs
    # the same requests all arriving at once: the server's capacity
    burst = [(0.0, kind, n, seed) for _, kind, n, seed in trace]
    sat, breqs, _, _ = form("fp64", budget, arrivals=burst)
    del breqs
    torch.cuda.empty_cache()
    out = base_line(args, plain["solves_per_s"], steps, warmup, plain["makespan_s"], plat,
                    "fp64")
    out["config"] = {
        "workload": f"served stream: {count} Poisson arrivals at {rate:.1f}/s (0.8 x the "
                    f"measured one-at-a-time capacity of {cap:.1f} solves/s unless set), sizes "
                    f"65^3/129^3/257^3/385^3 (p=.4/.3/.2/.1), quadratic or exp-cos, tol 1e-8, "
                    f"fp64, HBM budget {budget / 2**30:.1f} GiB, continuous batching, "
                    + (f"lanes {args.lanes}" if lanes else "one resident batch"),
        "requests": count, "rate_per_s": rate, "capacity_one_at_a_time_per_s": cap,
        "solo_ms": {str(n + 1): 1e3 * t for n, t in solo.items()},
        "budget_bytes": budget, "precision": "fp64", "lanes": args.lanes if lanes else None,
        "step": f"{STEP_REQUESTS} requests of the arrival trace",
        "latency": "completion - arrival",
        "request_data": "on the device before the clock starts (the client's payload)"}
    by_n = {}
    for n, rep in plain_reports:
        by_n.setdefault(n, []).append(rep)
    cyc = {n: (float(np.mean([r["init_cycles"] for r in reps])),
               float(np.mean([r["cycles"] for r in reps]))) for n, reps in by_n.items()}
    out.update({"forms": {"fp64": plain, "mixed": mixed}, "small_budget": small,
                "saturation": {"solves_per_s": sat["solves_per_s"], "p50_ms": sat["p50_ms"],
                               "p99_ms": sat["p99_ms"], "makespan_s": sat["makespan_s"],
                               "arrivals": "the same requests, all at t = 0",
                               "vs_one_at_a_time": sat["solves_per_s"] / cap},
                "chosen_form": "fp64",
                "updates_per_s": sum(r["point_updates"] for _, r in plain_reports)
                / plain["makespan_s"],
                "cycles_by_size": {str(n + 1): list(c) for n, c in cyc.items()},
                "roofline": served_roofline()})
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = served_cpu_baseline(cyc)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (the "
                                   "multi-GPU layout is documented as a design only)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.roofline_only:
        print(json.dumps({"roofline": served_roofline()}), flush=True)
        return
    precision = args.precision or ("mixed" if args.workload == "batch64" else "fp64")
    if args.workload in SINGLE:
        out = run_single(args, precision)
    elif args.workload in GS:
        out = run_gs(args, precision)
    elif args.workload in TWO_D:
        out = run_2d(args, precision)
    elif args.workload == "batch64":
        out = run_batch(args, precision)
    else:
        out = run_served(args, precision)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
