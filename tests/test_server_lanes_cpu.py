"""Size-class lanes of the serving loop (no GPU): one resident batch per
class, each ticking in its own thread; a fake backend whose tick costs real
(short) time that grows with the largest solve resident in that batch."""
import threading
import time

import numpy as np
import pytest

from paper_1411_7018_amd.server import Request, Server


class FakeBatch:
    def __init__(self, be, slots):
        self.be, self.slots, self.live = be, slots, {}

    def add(self, solver, u, f):
        free = [s for s in range(self.slots) if s not in self.live]
        assert free, "lane added beyond the slot limit"
        self.live[free[0]] = [self.be.ticks_for(solver["n"]), solver]
        return free[0]

    def tick(self):
        biggest = max(v[1]["n"] for v in self.live.values())
        time.sleep(self.be.tick_seconds(biggest))
        done = {}
        for s, v in self.live.items():
            v[0] -= 1
            if v[0] <= 0:
                done[s] = 1
        with self.be.lock:
            self.be.concurrent_now -= len(done)
        return done

    def report(self, slot):
        return {"cycles": self.be.ticks_for(self.live[slot][1]["n"])}

    def remove(self, slot):
        del self.live[slot]

    def close(self):
        pass


class FakeBackend:
    def __init__(self, slots=64):
        self.slots = slots
        self.lock = threading.Lock()
        self.concurrent_now = 0
        self.max_concurrent = 0
        self.streams = 0

    def hierarchy_bytes(self, n):
        return 5 * n ** 3

    def array_bytes(self, n):
        return 2 * n ** 3

    def ticks_for(self, n):
        return max(2, n // 16)

    def tick_seconds(self, n):
        return 2e-4 * (n / 16) ** 2

    def new_solver(self, n):
        return {"n": n}

    def data(self, req):
        return None, None

    def new_stream(self):
        with self.lock:
            self.streams += 1
        return object()

    def on_stream(self, stream):
        import contextlib
        return contextlib.nullcontext()

    def new_batch(self, stream=None):
        return FakeBatch(self, self.slots)

    def add(self, batch, solver, u, f):
        with self.lock:
            self.concurrent_now += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent_now)
        return batch.add(solver, u, f)


def reqs(spec):
    return [Request(i, t, "quadratic", n, i) for i, (t, n) in enumerate(spec)]


LANES = [[16], [32], [128]]


def test_lanes_serve_everything():
    be = FakeBackend()
    spec = [(0.001 * i, [16, 32, 128][i % 3]) for i in range(30)]
    rs = reqs(spec)
    st = Server(be, 10 ** 12, lanes=LANES).run(rs)
    assert st.completed == 30 and st.rejected == 0
    assert be.streams == 3
    for r in rs:
        assert r.status == 0 and r.report["cycles"] == be.ticks_for(r.n)


def test_small_requests_do_not_wait_on_large_ticks():
    """In one batch a small request ticks at the pace of the largest solve
    resident; with lanes it ticks at its own."""
    spec = [(0.0, 128)] + [(0.002 + 0.004 * i, 16) for i in range(10)]

    def small_p50(lanes):
        rs = reqs(spec)
        Server(FakeBackend(), 10 ** 12, lanes=lanes).run(rs)
        return float(np.median([r.latency for r in rs if r.n == 16]))

    one, many = small_p50(None), small_p50(LANES)
    assert many < 0.5 * one, (one, many)


def test_lanes_share_the_budget():
    be = FakeBackend()
    per = be.hierarchy_bytes(32) + be.array_bytes(32)
    spec = [(0.0, 32)] * 6 + [(0.0, 16)] * 6
    rs = reqs(spec)
    budget = 3 * per
    srv = Server(be, budget, lanes=LANES, pool=False)
    st = srv.run(rs)
    assert st.completed == 12
    assert st.peak_bytes <= budget
    assert srv.used == 0


def test_lanes_reject_oversized_and_serve_the_rest():
    be = FakeBackend()
    spec = [(0.0, 16), (0.0, 1024), (0.0, 32)]
    rs = reqs(spec)
    budget = 4 * (be.hierarchy_bytes(32) + be.array_bytes(32))
    st = Server(be, budget, lanes=LANES).run(rs)
    assert st.rejected == 1 and st.completed == 2
    assert rs[1].status == 2


def test_lane_errors_propagate():
    class Broken(FakeBackend):
        def new_batch(self, stream=None):
            b = FakeBatch(self, self.slots)

            def tick():
                raise RuntimeError("device lost")
            b.tick = tick
            return b

    with pytest.raises(RuntimeError, match="device lost"):
        Server(Broken(), 10 ** 12, lanes=LANES).run(reqs([(0.0, 16), (0.0, 32)]))
