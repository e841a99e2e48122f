#!/usr/bin/env python3
"""Benchmark of the FAS multigrid Monge-Ampere solver on one MI355X.

Default workload (one step = one complete solve): the 129^3 seeded quadratic
problem (u = x^T A x / 2 + b^T x, A SPD with eigenvalues in [0.5, 2],
f = det A): Poisson initial guess, then FAS V(2,2) cycles until the relative
discrete L2 residual is <= 1e-8, every input resident in HBM before timing
starts.  Other workloads:
  example4_17, expcos257, expcos385   single solves of other sizes;
  batch64   64 seeded solves (sizes 33^3..129^3, quadratic or exp-cos) run
            as one batch; one step = the whole batch;
  served    a Poisson-arrival stream of requests (65^3..385^3) through the
            continuous-batching server; --steps requests.
Before timing, the autotuner picks the engine's launch shapes on the same
solvers and data (outside the timed region; --no-tune keeps the defaults).

Prints one JSON line: solves/s (value), p50/p99 latency, grid-point
updates/s, the finest-level smoother's algorithmic bandwidth against the HBM
peak (HIP events around its launches inside the timed region), and, for the
default run, the CPU oracle timed on a bounded sample of the same workload.
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
# known size): profiles/k_batched_sweep_quadratic129_counters.md.  Valid for
# the k_batched sweep kernel as profiled; reset to None when it changes.
SERVE_RATE = 30.0   # served stream: Poisson arrivals per second
TRAFFIC = {("quadratic129", "fp64"): 31601357}
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
                    help="timed steps (served: requests); default per workload")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="quadratic129", choices=WORKLOADS)
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
    ap.add_argument("--rate", type=float, default=None,
                    help=f"served: arrivals per second (default {SERVE_RATE:g})")
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
           "kernel": "k_batched sweep, finest level (24 B per interior node per sweep)",
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


def retune_like(solvers, choice):
    """Give the instrumented solvers the launch shape the timed ones use."""
    if choice is not None:
        for s in solvers:
            s.retune(coarse_n=choice.coarse_n, max_blocks=choice.max_blocks,
                     strip_rows=choice.strip_rows, block_n=choice.block_n)


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
                "roofline": dict(roofline([reps[0] for reps in preps]),
                                 **instrumented(preps, tp, nsol))})
    return out


def run_served(args, precision):
    import torch

    from paper_1411_7018_amd import problems as P
    from paper_1411_7018_amd.server import GpuBackend, Server, requests_from_trace

    count = args.steps or 256
    warmup = 8 if args.warmup is None else args.warmup
    # a fixed arrival rate, below what one GPU serves of this size mix (about
    # 38 solves/s in FP64): the latencies then measure service and ordinary
    # queueing, not a queue that grows without bound
    rate = SERVE_RATE if args.rate is None else args.rate
    budget = int(args.budget_gb * (1 << 30)) if args.budget_gb else GpuBackend.budget_default()
    lanes = None
    if args.lanes and args.lanes != "none":
        # classes of grid sizes in points per side (65, 129, ...); requests carry n
        lanes = [[int(p) - 1 for p in c.split(",")] for c in args.lanes.split("/")]
    be = GpuBackend(precision=precision, tol=1e-8, max_slots=64)
    if warmup:
        Server(be, budget, lanes=lanes).run(
            requests_from_trace(P.arrival_trace(warmup, rate, seed=4999)))
    torch.cuda.synchronize()
    reqs = requests_from_trace(P.arrival_trace(count, rate, seed=5000))
    srv = Server(be, budget, max_slots=64, lanes=lanes)
    t0 = time.perf_counter()
    st = srv.run(reqs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat = [r.latency for r in reqs if r.status == 0]
    out = base_line(args, st.solves_per_s, count, warmup, elapsed, lat, precision)
    out["config"] = {
        "workload": f"served stream: {count} Poisson arrivals at {rate:.1f}/s, sizes "
                    f"65^3/129^3/257^3/385^3 (p=.4/.3/.2/.1), quadratic or exp-cos, tol 1e-8, "
                    f"{precision}, HBM budget {budget / 2**30:.1f} GiB, continuous batching, "
                    + (f"lanes {args.lanes}" if lanes else "one resident batch"),
        "requests": count, "rate_per_s": rate, "budget_bytes": budget, "precision": precision,
        "lanes": args.lanes if lanes else None,
        "latency": "completion - arrival"}
    out.update({"completed": st.completed, "rejected": st.rejected,
                "mean_live": st.mean_live, "max_live": st.max_live, "queued": st.queued,
                "peak_bytes": st.peak_bytes, "ticks": st.ticks,
                "updates_per_s": sum(r.report["point_updates"] for r in reqs if r.report)
                / st.makespan})
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
