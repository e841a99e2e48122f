"""The z-stream sweep (all four colour phases of a sweep in one launch, each
workgroup walking a column of the grid plane by plane with the phases two
planes apart, out of place) at the sizes it is built for: bitwise equal to
the colour-phase kernels over pairs of sweeps at 129^3, 257^3 and 385^3.
The colour-phase form is itself checked node by node against the oracle at
these sizes (test_gpu_fullsize), and the engine's V-cycle with z-stream
sweeps on its finest level against the oracle's V-cycle (test_gpu_benchshape)."""
import sys

import numpy as np
import pytest

from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ZS_CONFIGS = (8, 9, 10, 11, 12)


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def solver(n, **kw):
    from paper_1411_7018_amd import Solver
    return Solver(n, **kw)


@pytest.mark.parametrize("n", [128, 256, 384])
def test_zsweep_full_size_bitwise_vs_colour(n):
    note("z-stream sweep full size", n)
    u0, f, ue = P.make_device("exp_cos", n, 7000 + n, exact=True)
    # a smooth convex start: the solution plus a bump that vanishes on the boundary
    t = torch.arange(n + 1, dtype=torch.float64, device="cuda") / n
    s = torch.sin(np.pi * t)
    start = ue + 0.01 * s[:, None, None] * s[None, :, None] * s[None, None, :]
    del ue
    uc = start.clone()
    solver(n, smoother="color").sweep(uc, f, 2)
    for cfg in ZS_CONFIGS:
        uz = start.clone()
        solver(n, smoother="fused", tile_config=cfg).sweep(uz, f, 2)
        torch.cuda.synchronize()
        assert torch.equal(uz, uc), cfg
        del uz


def _solve(n, kind, seed, **kw):
    s = solver(n, **kw)
    u0, f = P.make_device(kind, n, seed)
    u = u0.clone()
    rep = s.solve(u, f, tol=1e-9)
    torch.cuda.synchronize()
    return u.cpu().numpy(), rep


@pytest.mark.parametrize("n,kind,kw", [
    (256, "exp_cos", {}),                                   # automatic: finest level only
    (224, "exp_cos", {}),                                   # automatic, ragged columns and chunks
    (128, "quadratic", {"smoother": "fused", "tile_config": 8}),
    (96, "exp_cos", {"smoother": "fused", "tile_config": 9}),
    (128, "exp_cos", {"smoother": "fused", "tile_config": 10}),
    (64, "exp_cos", {"smoother": "fused", "tile_config": 11}),
    (160, "exp_cos", {"smoother": "fused", "tile_config": 12}),  # one colour per wavefront
])
def test_fused_prolongation_solve_bitwise(n, kind, kw):
    """Solves whose first post-smoothing z-stream sweep also applies the
    coarse-grid correction (no separate prolongation pass) equal, bitwise
    and in cycle count, the same solves with the separate pass and with
    colour phases everywhere."""
    note("fused prolongation solve", n, kind, kw)
    uf, rf = _solve(n, kind, 8100 + n, **kw)
    us, rs = _solve(n, kind, 8100 + n, fuse_prolong=-1, **kw)
    uc, rc = _solve(n, kind, 8100 + n, smoother="color")
    assert rf["cycles"] == rs["cycles"] == rc["cycles"]
    assert np.array_equal(uf, us)
    assert np.array_equal(uf, uc)


def test_fused_prolongation_batch_bitwise():
    """A batch of different sizes, z-stream sweeps on every multi-block
    level: each solve's result is that of colour phases."""
    from paper_1411_7018_amd.batch import solve_batch
    specs = [("quadratic", 128, 1), ("exp_cos", 64, 2), ("example4", 96, 3), ("exp_cos", 48, 4)]
    note("fused prolongation batch")
    res = {}
    for mode in ("color", "zs"):
        kw = {"smoother": "color"} if mode == "color" else {"smoother": "fused", "tile_config": 8}
        solvers, us, fs = [], [], []
        for kind, n, seed in specs:
            u0, f = P.make_device(kind, n, seed)
            solvers.append(solver(n, **kw))
            us.append(u0)
            fs.append(f)
        st, reps = solve_batch(solvers, us, fs, tol=1e-9)
        assert st == 0
        torch.cuda.synchronize()
        res[mode] = ([u.cpu().numpy() for u in us], [r["cycles"] for r in reps])
    assert res["zs"][1] == res["color"][1]
    for a, c in zip(res["zs"][0], res["color"][0]):
        assert np.array_equal(a, c)
