"""Continuous-batching server on the GPU: requests that arrive while others
are cycling join the resident batch; every result equals (bitwise) the same
request solved alone, for the plain FP64 and the mixed-precision form, with
a roomy budget and with one that forces admission queueing, with one
resident batch and with one batch per size class (lanes ticking on their
own streams from their own threads)."""
import sys

import numpy as np
import pytest

from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def trace(count=10, seed=77):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(0.002)
        kind = "quadratic" if rng.random() < 0.5 else "exp_cos"
        out.append((t, kind, int(rng.choice([16, 24, 32, 48])), 900 + i))
    return out


def solo(kind, n, seed, precision):
    from paper_1411_7018_amd import Solver
    u, f = P.make_device(kind, n, seed)
    Solver(n, precision=precision).solve(u, f, tol=1e-8)
    torch.cuda.synchronize()
    return u.cpu().numpy()


LANES = [[16, 24], [32], [48]]


@pytest.mark.parametrize("precision,tight,lanes", [("fp64", False, None), ("mixed", False, None),
                                                   ("fp64", True, None), ("fp64", False, LANES),
                                                   ("mixed", False, LANES), ("fp64", True, LANES)])
def test_served_results_equal_solo(precision, tight, lanes):
    from paper_1411_7018_amd.server import GpuBackend, Server, requests_from_trace
    note("server", precision, "tight" if tight else "roomy", "lanes" if lanes else "one batch")
    be = GpuBackend(precision=precision, tol=1e-8, max_slots=8)
    reqs = requests_from_trace(trace())
    if tight:
        big = max(r.n for r in reqs)
        budget = be.hierarchy_bytes(big) + be.array_bytes(big) + be.hierarchy_bytes(16) \
            + be.array_bytes(16)
    else:
        budget = 8 << 30
    srv = Server(be, budget, max_slots=8, keep_results=True, lanes=lanes)
    st = srv.run(reqs)
    assert st.completed == len(reqs) and st.rejected == 0
    assert srv.peak <= budget
    if not tight:
        assert st.max_live > 1
    elif lanes is None:
        assert st.queued >= 1
    for r in reqs:
        assert r.status == 0
        want = solo(r.kind, r.n, r.seed, precision)
        assert np.array_equal(r.u.cpu().numpy(), want), (r.rid, r.kind, r.n)


def oracle_trace():
    """Requests of the served stream's smaller sizes (65^3, 129^3) beside
    small ones, arriving while others cycle."""
    sizes = [64, 32, 128, 64, 16, 64]
    kinds = ["exp_cos", "quadratic", "exp_cos", "quadratic", "exp_cos", "exp_cos"]
    return [(0.003 * i, kinds[i], sizes[i], 5100 + i) for i in range(len(sizes))]


@pytest.mark.parametrize("lanes", [None, [[16, 32, 64], [128]]])
def test_served_fp64_results_match_oracle(lanes):
    """Each served FP64 result equals the oracle's solve of the same data
    (Poisson guess, FAS V(2,2) to 1e-8) at the same cycle count, to 1e-12."""
    import oracle
    from paper_1411_7018_amd.server import GpuBackend, Server, requests_from_trace
    note("server vs oracle fp64", "lanes" if lanes else "one batch")
    be = GpuBackend(precision="fp64", tol=1e-8, max_slots=8)
    reqs = requests_from_trace(oracle_trace())
    srv = Server(be, 8 << 30, max_slots=8, keep_results=True, lanes=lanes)
    st = srv.run(reqs)
    assert st.completed == len(reqs) and st.max_live > 1
    for r in reqs:
        u0, f = P.make_device(r.kind, r.n, r.seed)
        torch.cuda.synchronize()
        want = u0.cpu().numpy()
        ost, orep, _ = oracle.solve(want, f.cpu().numpy(), oracle.params(tol=1e-8))
        assert ost == 0
        assert r.status == 0 and r.report["cycles"] == orep.cycles, (r.rid, r.n)
        got = r.u.cpu().numpy()
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), (r.rid, r.kind, r.n)


@pytest.mark.parametrize("tol,bound", [(1e-10, 1e-10), (1e-8, 1e-8)])
def test_served_mixed_results_match_oracle_limit(tol, bound):
    """Each served mixed-precision result against the oracle's converged
    discrete solution (run to its round-off floor): <= 1e-10 in the max norm
    when the stream runs to 1e-10; at the 1e-8 stop the remaining solver
    error is of order ||L^-1|| * 1e-8 and the agreement reached is printed."""
    import oracle
    from paper_1411_7018_amd.server import GpuBackend, Server, requests_from_trace
    note("server vs oracle limit mixed", tol)
    be = GpuBackend(precision="mixed", tol=tol, max_slots=8)
    reqs = requests_from_trace([x for x in oracle_trace() if x[2] <= 64])
    srv = Server(be, 8 << 30, max_slots=8, keep_results=True)
    st = srv.run(reqs)
    assert st.completed == len(reqs)
    worst = 0.0
    for r in reqs:
        u0, f = P.make_device(r.kind, r.n, r.seed)
        torch.cuda.synchronize()
        lim = u0.cpu().numpy()
        oracle.solve_limit(lim, f.cpu().numpy())
        d = float(np.abs(r.u.cpu().numpy() - lim).max())
        worst = max(worst, d)
        assert r.status == 0 and d <= bound, (r.rid, r.kind, r.n, d)
    note(f"served mixed at tol {tol:g}: max|u - oracle limit| = {worst:.3e}")
