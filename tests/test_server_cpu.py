"""Scheduling logic of the continuous-batching server (no GPU): a fake
backend whose solves need a size-dependent number of ticks, and a simulated
clock advanced by each tick's cost."""
import pytest

from paper_1411_7018_amd.server import Request, Server


class FakeBatch:
    def __init__(self, backend, slots):
        self.be = backend
        self.slots = slots
        self.live = {}

    def add(self, solver, u, f):
        free = [s for s in range(self.slots) if s not in self.live]
        assert free, "server added beyond the slot limit"
        s = free[0]
        self.live[s] = [self.be.ticks_for(solver["n"]), solver]
        self.be.max_concurrent = max(self.be.max_concurrent, len(self.live))
        return s

    def tick(self):
        self.be.clock.t += self.be.tick_cost(len(self.live))
        done = {}
        for s, v in self.live.items():
            v[0] -= 1
            if v[0] <= 0:
                done[s] = 2 if v[1]["n"] in self.be.fail else 1
        return done

    def report(self, slot):
        n = self.live[slot][1]["n"]
        return {"cycles": self.be.ticks_for(n), "res": self.be.fail.get(n, 1e-9)}

    def remove(self, slot):
        del self.live[slot]

    def close(self):
        pass


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeBackend:
    def __init__(self, slots=64):
        self.clock = Clock()
        self.slots = slots
        self.max_concurrent = 0
        self.solvers_made = 0
        self.fail = {}      # n -> final residual of a solve of that size that fails

    def hierarchy_bytes(self, n):
        return 5 * n ** 3

    def array_bytes(self, n):
        return 2 * n ** 3

    def ticks_for(self, n):
        return max(2, n // 16)

    def tick_cost(self, live):
        return 1e-3 * (1 + live)

    def new_solver(self, n):
        self.solvers_made += 1
        return {"n": n}

    def data(self, req):
        return None, None

    def new_batch(self):
        return FakeBatch(self, self.slots)

    def add(self, batch, solver, u, f):
        return batch.add(solver, u, f)


def run(reqs, budget, slots=64, fail=None, **kw):
    be = FakeBackend(slots)
    be.fail = fail or {}
    srv = Server(be, budget, max_slots=slots, **kw)
    # wrap the memory accounting to check the budget after every admission
    orig = srv._try_admit

    def checked(req):
        v = orig(req)
        assert srv.used <= srv.budget
        return v

    srv._try_admit = checked
    st = srv.run(reqs, clock=be.clock, sleep=be.clock.sleep)
    return st, srv, be


def trace(sizes, gap):
    return [Request(i, i * gap, "k", n, i) for i, n in enumerate(sizes)]


def test_all_served_and_overlapping():
    reqs = trace([16, 32, 64, 16, 32, 64, 16, 48], gap=0.002)
    st, srv, be = run(reqs, budget=10 ** 9)
    assert st.completed == len(reqs) and st.rejected == 0
    assert be.max_concurrent > 1                      # continuous batching
    for r in reqs:
        assert r.status == 0 and r.t_admit >= r.t_arrival and r.t_done > r.t_admit
    # a request that arrives while others run is admitted before they finish
    assert any(r.t_admit < max(q.t_done for q in reqs[:i]) for i, r in enumerate(reqs) if i)


def test_slot_limit():
    reqs = trace([16] * 20, gap=0.0)
    st, srv, be = run(reqs, budget=10 ** 9, slots=3)
    assert st.completed == 20 and be.max_concurrent == 3 and st.max_live == 3


def test_budget_forces_queueing_in_arrival_order():
    sizes = [64] * 6
    per = 7 * 64 ** 3
    reqs = trace(sizes, gap=0.0)
    st, srv, be = run(reqs, budget=2 * per)
    assert st.completed == 6
    assert be.max_concurrent == 2 and srv.peak <= 2 * per
    admits = [r.t_admit for r in reqs]
    assert admits == sorted(admits)                    # first come first served
    assert st.queued >= 3


def test_oversized_request_rejected_others_served():
    reqs = trace([16, 128, 16], gap=0.001)
    st, srv, be = run(reqs, budget=7 * 64 ** 3)
    assert st.completed == 2 and st.rejected == 1
    assert reqs[1].status == 2 and reqs[0].status == 0 and reqs[2].status == 0


def test_pool_reuses_hierarchies():
    reqs = trace([32] * 10, gap=0.05)              # each finishes before the next
    st, srv, be = run(reqs, budget=10 ** 9)
    assert st.completed == 10 and be.solvers_made == 1
    st2, srv2, be2 = run(trace([32] * 10, gap=0.05), budget=10 ** 9, pool=False)
    assert be2.solvers_made == 10 and srv2.used == 0


def test_idle_pool_is_evicted_to_admit():
    # a 64 leaves its idle hierarchy behind; a later 96 only fits once it goes
    reqs = trace([64, 96], gap=0.5)
    budget = 7 * 96 ** 3
    st, srv, be = run(reqs, budget=budget)
    assert st.completed == 2
    assert srv.peak <= budget


def test_skip_ahead_lets_small_requests_pass():
    big, small = 96, 16
    budget = 7 * 96 ** 3 + 7 * small ** 3
    sizes = [96, 96, 16, 16, 16]
    fifo = run(trace(sizes, gap=0.0), budget)[0]
    skip_reqs = trace(sizes, gap=0.0)
    skip = run(skip_reqs, budget, skip_ahead=True)[0]
    assert fifo.completed == skip.completed == 5
    # with skip-ahead the small ones start before the second big one
    assert skip_reqs[2].t_admit < skip_reqs[1].t_admit


def test_stats_percentiles():
    reqs = trace([16] * 50, gap=0.01)
    st, _, _ = run(reqs, budget=10 ** 9)
    lat = sorted(r.latency for r in reqs)
    assert st.p50 == pytest.approx(lat[24] / 2 + lat[25] / 2)
    assert st.p99 >= st.p50 > 0 and st.solves_per_s > 0


def test_failed_solves_keep_their_own_status():
    """A solve that stops with an error is reported as not converged or
    non-finite, never as the rejection status of admission."""
    from paper_1411_7018_amd.server import (MA_ERR_NONFINITE, MA_ERR_NOT_CONVERGED,
                                            MA_ERR_OOM)
    reqs = trace([16, 32, 48, 16, 128], gap=0.001)
    st, srv, be = run(reqs, budget=7 * 64 ** 3, fail={32: 3.0, 48: float("nan")})
    assert [r.status for r in reqs] == [0, MA_ERR_NOT_CONVERGED, MA_ERR_NONFINITE, 0,
                                       MA_ERR_OOM]
    assert st.completed == 2 and st.rejected == 1
