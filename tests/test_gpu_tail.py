"""The coarse end of the V-cycle in one workgroup per solve (k_tail, and its
LDS form when the coarse levels fit in LDS): a solve gives the same bits and
cycle counts whatever levels the coarse-level kernel takes over (coarse_n 0:
none; 8 and 16: the LDS form; 32: the global-memory form), for both
orderings, both restrictions, both precisions and in batches."""
import sys

import numpy as np
import pytest

from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run(n, kind, seed, coarse_n, tol=1e-9, **kw):
    """A full solve; with half-weighting (which with multicolour smoothing
    does not converge on these problems) three V-cycles from the Poisson
    start instead."""
    from paper_1411_7018_amd import Solver
    p = P.make(kind, n, seed)
    s = Solver(n, coarse_n=coarse_n, **kw)
    u, f = dev(P.initial_guess(p)), dev(p.f)
    if kw.get("restriction") == "half":
        s.poisson_init(u, f)
        for _ in range(3):
            s.vcycle(u, f)
        rep = {"cycles": 3, "nonconvex": 0}
    else:
        rep = s.solve(u, f, tol=tol)
    s.close()
    return host(u), rep


CASES = [(16, "quadratic", 1, {}), (32, "exp_cos", 2, {}), (64, "example4", 3, {}),
         (128, "exp_cos", 4, {}), (96, "quadratic", 5, {}), (40, "exp_cos", 6, {}),
         (64, "exp_cos", 7, {"order": "8c"}), (64, "example4", 8, {"restriction": "half"}),
         (48, "exp_cos", 9, {"precision": "mixed"})]


@pytest.mark.parametrize("n,kind,seed,kw", CASES)
def test_coarse_n_same_bits(n, kind, seed, kw):
    note("tail", n, kind, kw)
    u0, r0 = run(n, kind, seed, 0, **kw)
    for cn in (8, 16, 32):
        u, r = run(n, kind, seed, cn, **kw)
        assert r["cycles"] == r0["cycles"], cn
        assert r["nonconvex"] == r0["nonconvex"], cn
        assert np.array_equal(u, u0), cn


def test_batch_tail_forms_same_bits():
    from paper_1411_7018_amd import Solver
    from paper_1411_7018_amd.batch import solve_batch
    specs = [("quadratic", 128, 1), ("exp_cos", 64, 2), ("example4", 16, 3), ("exp_cos", 40, 4),
             ("quadratic", 8, 5)]
    note("batch tail")
    out = {}
    for cn in (0, 16):
        solvers, us, fs = [], [], []
        for kind, n, seed in specs:
            p = P.make(kind, n, seed)
            solvers.append(Solver(n, coarse_n=cn))
            us.append(dev(P.initial_guess(p)))
            fs.append(dev(p.f))
        st, reps = solve_batch(solvers, us, fs, tol=1e-9)
        assert st == 0
        out[cn] = ([host(u) for u in us], [r["cycles"] for r in reps])
    assert out[0][1] == out[16][1]
    for a, b in zip(out[0][0], out[16][0]):
        assert np.array_equal(a, b)
