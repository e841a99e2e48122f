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
