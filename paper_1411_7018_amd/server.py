"""Continuous-batching server for Monge-Ampere solve requests.

Requests arrive over time (e.g. ``problems.arrival_trace``: Poisson
arrivals, grid sizes 65^3 .. 385^3).  The server keeps ONE resident batch
(``ma_batch``): every tick advances each admitted solve by one step (a
linear V-cycle of its Poisson initial guess, then FAS V-cycles, batched by
level on the device).  Between ticks it

  * retires the solves that finished (converged or failed), and
  * admits queued requests while a slot is free and the HBM footprint of the
    new solve -- its multigrid hierarchy plus its u and f arrays -- fits the
    budget next to everything already resident.

Hierarchies are kept after their request leaves (a per-size pool of idle
solvers), so a later request of the same size allocates nothing; idle
solvers are evicted, least recently used first, when a new request would
not fit otherwise.  Admission is first-come first-served; with
``skip_ahead`` a request that does not fit yet lets smaller ones behind it
start.  A request larger than the whole budget is rejected (status
MA_ERR_OOM) and the rest are still served.

With ``lanes`` the server keeps one resident batch per size class
instead, each ticking on its own stream from its own host thread, so a small
request advances at the pace of its own class rather than in lock step with
the largest solve resident; the lanes share the HBM budget and the pool of
idle hierarchies.

Each solve's arithmetic and stopping decisions are its own (the engine
batches launches, never data), so a result is bitwise the same alone and in
any mix.  The scheduling logic talks to a small backend interface, so it
runs unchanged on the GPU (``GpuBackend``) and under a simulated clock in
CPU tests.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time

import numpy as np

# ma_status values (include/ma.h)
MA_ERR_OOM = 2
MA_ERR_NOT_CONVERGED = 4
MA_ERR_NONFINITE = 5


def failure_status(report) -> int:
    """Status of a solve that left the batch with an error (ma_batch_tick
    marks it 2): a residual norm that is not finite, else the cycle limit.
    Distinct from MA_ERR_OOM, which the server gives to rejected requests."""
    res = (report or {}).get("res")
    if res is not None and not math.isfinite(res):
        return MA_ERR_NONFINITE
    return MA_ERR_NOT_CONVERGED


@dataclasses.dataclass
class Request:
    rid: int
    t_arrival: float          # seconds after the start of the run
    kind: str
    n: int
    seed: int
    t_admit: float | None = None
    t_done: float | None = None
    status: int | None = None   # 0 converged, else an ma_status
    report: dict | None = None
    u: object = None            # the solution (kept when keep_results)
    payload: object = None      # (u0, f) already on the device, or None: made on admission

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class GpuBackend:
    """Solvers, request data and the resident batch on the current GPU."""

    def __init__(self, precision: str = "fp64", tol: float = 1e-8, max_slots: int = 64,
                 **params):
        from .solver import footprint_bytes

        self.precision = precision
        self.tol = tol
        self.params = params
        self.max_slots = max_slots
        self._fp = footprint_bytes
        self._hier = {}

    def hierarchy_bytes(self, n: int) -> int:
        if n not in self._hier:
            self._hier[n] = int(self._fp(n, precision=self.precision, **self.params))
        return self._hier[n]

    def array_bytes(self, n: int) -> int:
        return 2 * (n + 1) ** 3 * 8            # u and f, FP64

    def new_solver(self, n: int):
        from .solver import Solver

        return Solver(n, precision=self.precision, **self.params)

    def data(self, req: Request):
        """The request's (u, f): its payload when the client has put it on
        the device already, else made now on the current stream."""
        if req.payload is not None:
            u, f = req.payload
            req.payload = None
            return u, f
        from .problems import make_device

        return make_device(req.kind, req.n, req.seed)

    def new_batch(self, stream=None):
        from .batch import ResidentBatch

        return ResidentBatch(self.max_slots, stream=stream)

    def new_stream(self):
        import torch

        return torch.cuda.Stream()

    def on_stream(self, stream):
        """Context in which the calls of a lane's thread order their work on
        the lane's stream (request data included)."""
        import torch

        return torch.cuda.stream(stream)

    def add(self, batch, solver, u, f) -> int:
        return batch.add(solver, u, f, tol=self.tol)

    @staticmethod
    def budget_default(reserve: float = 0.1) -> int:
        import torch

        free, _ = torch.cuda.mem_get_info()
        return int(free * (1.0 - reserve))


@dataclasses.dataclass
class Stats:
    completed: int
    rejected: int
    makespan: float
    p50: float
    p99: float
    mean: float
    solves_per_s: float
    max_live: int
    mean_live: float
    peak_bytes: int
    ticks: int
    queued: int                 # requests admitted more than 1 ms after arrival

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


class Server:
    def __init__(self, backend, budget_bytes: int, max_slots: int = 64, pool: bool = True,
                 skip_ahead: bool = False, keep_results: bool = False, lanes=None):
        """lanes: None (one batch for all sizes) or a list of size classes,
        each a collection of grid sizes n; a size in no class joins the
        last one.  max_slots bounds each lane's batch."""
        if not 1 <= max_slots <= 64:
            raise ValueError("max_slots must be in 1..64")
        self.lanes = [frozenset(int(n) for n in c) for c in lanes] if lanes else None
        if self.lanes is not None and not self.lanes:
            raise ValueError("lanes must name at least one size class")
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.pool = pool
        self.skip_ahead = skip_ahead
        self.keep_results = keep_results
        self.used = 0                    # resident hierarchies + live arrays
        self.peak = 0
        self.idle = collections.OrderedDict()   # (n, serial) -> solver, LRU first
        self._serial = 0
        self.created = 0                 # solvers allocated
        self.batch = None

    # -- memory -----------------------------------------------------------
    def _evict_one(self, protect) -> bool:
        """Free the least recently used idle hierarchy other than protect."""
        for k in self.idle:
            if k != protect:
                self.idle.pop(k)
                self.used -= self.be.hierarchy_bytes(k[0])
                return True
        return False

    def _try_admit(self, req: Request) -> str:
        """'ok', 'wait' or 'reject'."""
        n = req.n
        arrays = self.be.array_bytes(n)
        hier = self.be.hierarchy_bytes(n)
        if arrays + hier > self.budget:
            return "reject"
        reuse = next((k for k in self.idle if k[0] == n), None)
        need = arrays + (0 if reuse else hier)
        while self.used + need > self.budget and self._evict_one(reuse):
            pass
        if self.used + need > self.budget:
            return "wait"
        if reuse:
            solver = self.idle.pop(reuse)
        else:
            solver = self.be.new_solver(n)
            self.created += 1
        self.used += need
        self.peak = max(self.peak, self.used)
        u, f = self.be.data(req)
        slot = self.be.add(self.batch, solver, u, f)
        self._live[slot] = (req, solver, u, f)
        return "ok"

    # -- main loop --------------------------------------------------------
    def run(self, requests, clock=time.perf_counter, sleep=time.sleep) -> Stats:
        if self.lanes is not None and len(self.lanes) > 1:
            return self._run_lanes(requests, clock, sleep)
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        pending = collections.deque(reqs)
        queue = collections.deque()
        self._live = {}
        self.batch = self.be.new_batch()
        ticks, live_sum, max_live, queued = 0, 0, 0, 0
        rejected = 0
        t0 = clock()
        try:
            while pending or queue or self._live:
                now = clock() - t0
                while pending and pending[0].t_arrival <= now:
                    queue.append(pending.popleft())
                # admission, first come first served
                blocked = []
                while queue and len(self._live) < self.max_slots:
                    req = queue[0]
                    verdict = self._try_admit(req)
                    if verdict == "wait":
                        if not self.skip_ahead:
                            break
                        blocked.append(queue.popleft())
                        continue
                    queue.popleft()
                    if verdict == "reject":
                        req.status, req.t_admit, req.t_done = MA_ERR_OOM, now, now
                        rejected += 1
                        continue
                    req.t_admit = now
                    if req.t_admit > req.t_arrival + 1e-3:
                        queued += 1
                queue.extendleft(reversed(blocked))
                if self._live:
                    done = self.batch.tick()
                    ticks += 1
                    live_sum += len(self._live)
                    max_live = max(max_live, len(self._live))
                    tnow = clock() - t0
                    for slot, code in done.items():
                        req, solver, u, f = self._live.pop(slot)
                        req.report = self.batch.report(slot)
                        req.status = 0 if code == 1 else failure_status(req.report)
                        req.t_done = tnow
                        if self.keep_results:
                            req.u = u
                        self.batch.remove(slot)
                        self.used -= self.be.array_bytes(req.n)
                        if self.pool:
                            self._serial += 1
                            self.idle[(req.n, self._serial)] = solver
                        else:
                            self.used -= self.be.hierarchy_bytes(req.n)
                elif pending:
                    sleep(max(0.0, pending[0].t_arrival - (clock() - t0)))
                elif queue:
                    # nothing live and the head cannot be admitted: only
                    # idle hierarchies can be in the way, and eviction has
                    # already been tried, so the request can never fit
                    req = queue.popleft()
                    req.status, req.t_admit, req.t_done = MA_ERR_OOM, now, now
                    rejected += 1
        finally:
            self.batch.close()
            self.batch = None
        return self._stats(reqs, ticks, live_sum, max_live, rejected, queued)

    def _stats(self, reqs, ticks, live_sum, max_live, rejected, queued) -> Stats:
        done = [r for r in reqs if r.status == 0]
        lat = np.array([r.latency for r in done]) if done else np.zeros(1)
        t_first = reqs[0].t_arrival if reqs else 0.0
        t_last = max((r.t_done for r in done), default=t_first)
        makespan = max(t_last - t_first, 1e-12)
        return Stats(completed=len(done), rejected=rejected, makespan=makespan,
                     p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                     mean=float(lat.mean()), solves_per_s=len(done) / makespan,
                     max_live=max_live, mean_live=live_sum / max(ticks, 1),
                     peak_bytes=self.peak, ticks=ticks, queued=queued)


    # -- lanes ------------------------------------------------------------
    def _lane_of(self, n: int) -> int:
        for i, c in enumerate(self.lanes):
            if n in c:
                return i
        return len(self.lanes) - 1

    def _reserve(self, req: Request):
        """Admission decision under the lock: ("ok", reused solver or None),
        ("wait", None) or ("reject", None).  Budget and pool are updated
        here; the solver and the data are made by the lane afterwards."""
        n = req.n
        arrays = self.be.array_bytes(n)
        hier = self.be.hierarchy_bytes(n)
        if arrays + hier > self.budget:
            return "reject", None
        reuse = next((k for k in self.idle if k[0] == n), None)
        need = arrays + (0 if reuse else hier)
        while self.used + need > self.budget and self._evict_one(reuse):
            pass
        if self.used + need > self.budget:
            return "wait", None
        self.used += need
        self.peak = max(self.peak, self.used)
        if reuse:
            return "ok", self.idle.pop(reuse)
        self.created += 1
        return "ok", None

    def _run_lanes(self, requests, clock, sleep) -> Stats:
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        nl = len(self.lanes)
        cv = threading.Condition()
        queues = [collections.deque() for _ in range(nl)]
        live_count = [0] * nl
        arrived = {"all": False}
        counts = {"ticks": 0, "live_sum": 0, "max_live": 0, "rejected": 0, "queued": 0}
        errors = []
        t0 = clock()

        def lane(li):
            stream = self.be.new_stream()
            with self.be.on_stream(stream):
                batch = self.be.new_batch(stream)
                live = {}
                try:
                    while True:
                        admitted = []
                        with cv:
                            now = clock() - t0
                            q = queues[li]
                            while q and len(live) + len(admitted) < self.max_slots:
                                verdict, solver = self._reserve(q[0])
                                if verdict == "wait":
                                    # nothing live anywhere: only idle hierarchies
                                    # could be in the way, and they were evicted
                                    if not any(live_count) and not live and not admitted:
                                        verdict = "reject"
                                    else:
                                        break
                                req = q.popleft()
                                if verdict == "reject":
                                    req.status, req.t_admit, req.t_done = MA_ERR_OOM, now, now
                                    counts["rejected"] += 1
                                    continue
                                req.t_admit = now
                                if req.t_admit > req.t_arrival + 1e-3:
                                    counts["queued"] += 1
                                admitted.append((req, solver))
                            live_count[li] = len(live) + len(admitted)
                            if not live and not admitted:
                                if arrived["all"] and not q:
                                    return
                                cv.wait(0.005)
                                continue
                        for req, solver in admitted:
                            if solver is None:
                                solver = self.be.new_solver(req.n)
                            u, f = self.be.data(req)
                            slot = self.be.add(batch, solver, u, f)
                            live[slot] = (req, solver, u, f)
                        done = batch.tick()
                        tnow = clock() - t0
                        retired = []
                        for slot, code in done.items():
                            req, solver, u, f = live.pop(slot)
                            req.report = batch.report(slot)
                            req.status = 0 if code == 1 else failure_status(req.report)
                            req.t_done = tnow
                            if self.keep_results:
                                req.u = u
                            batch.remove(slot)
                            retired.append((req, solver))
                        with cv:
                            counts["ticks"] += 1
                            counts["live_sum"] += len(live) + len(retired)
                            counts["max_live"] = max(counts["max_live"],
                                                     sum(live_count))
                            for req, solver in retired:
                                self.used -= self.be.array_bytes(req.n)
                                if self.pool:
                                    self._serial += 1
                                    self.idle[(req.n, self._serial)] = solver
                                else:
                                    self.used -= self.be.hierarchy_bytes(req.n)
                            live_count[li] = len(live)
                            cv.notify_all()
                except BaseException as e:       # surfaced by run()
                    with cv:
                        errors.append(e)
                        arrived["all"] = True
                        cv.notify_all()
                finally:
                    batch.close()

        threads = [threading.Thread(target=lane, args=(i,), daemon=True) for i in range(nl)]
        for t in threads:
            t.start()
        try:
            for req in reqs:
                wait = req.t_arrival - (clock() - t0)
                if wait > 0:
                    sleep(wait)
                with cv:
                    if errors:
                        break
                    queues[self._lane_of(req.n)].append(req)
                    cv.notify_all()
        finally:
            with cv:
                arrived["all"] = True
                cv.notify_all()
            for t in threads:
                t.join()
        if errors:
            raise errors[0]
        return self._stats(reqs, counts["ticks"], counts["live_sum"], counts["max_live"],
                           counts["rejected"], counts["queued"])


def requests_from_trace(trace) -> list:
    """``problems.arrival_trace`` tuples -> Request objects."""
    return [Request(i, t, kind, n, seed) for i, (t, kind, n, seed) in enumerate(trace)]
