"""The block sweep (all four colour phases of a sweep in one launch, each
workgroup updating a block of the grid with its halo in LDS, out of place)
against the per-colour kernel (bitwise: the same point update on the same
neighbour values) and against the oracle (<= 1e-12 relative); and the
engine's use of it on the mid-size levels of the V-cycle: solves and batches
are bitwise the same whichever levels take block sweeps."""
import sys

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-12


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


def solver(n, **kw):
    from paper_1411_7018_amd import Solver
    return Solver(n, **kw)


def start(p, seed):
    rng = np.random.default_rng(seed)
    return P.initial_guess(p, p.u_exact * (1.0 + 1e-3 * rng.standard_normal(p.u_exact.shape)))


# ragged grids (n - 1 not a multiple of the block sides) and tiny ones;
# configurations 8..12 are the z-stream sweeps
@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12])
@pytest.mark.parametrize("n", [2, 4, 9, 33, 47, 64, 100])
def test_block_sweep_bitwise_vs_color_and_oracle(n, cfg):
    note("block sweep", n, cfg)
    p = P.exp_cos(n, seed=n + cfg)
    u0 = start(p, cfg)
    f = dev(p.f)
    uc = dev(u0)
    solver(n, smoother="color").sweep(uc, f, 2)
    ub = dev(u0)
    solver(n, smoother="fused", tile_config=cfg).sweep(ub, f, 2)
    got, ref = host(ub), host(uc)
    assert np.array_equal(got, ref)
    want = u0.copy()
    oracle.sweep(want, p.f, "4c")
    oracle.sweep(want, p.f, "4c")
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()


@pytest.mark.parametrize("count", [1, 3, 4])
def test_block_sweep_counts(count):
    """Pairs of sweeps run as block sweeps, an odd last one per colour."""
    n = 40
    note("block sweep count", count)
    p = P.example4(n)
    u0 = start(p, 7)
    f = dev(p.f)
    uc, ub = dev(u0), dev(u0)
    solver(n, smoother="color").sweep(uc, f, count)
    solver(n, smoother="fused").sweep(ub, f, count)
    assert np.array_equal(host(ub), host(uc))


@pytest.mark.parametrize("n", [40, 64])
def test_block_poisson_init_parity(n):
    note("block poisson", n)
    p = P.example4(n)
    want = P.initial_guess(p)
    oracle.poisson_init(want, p.f, oracle.params(init_tol=0.0, init_max_cycles=3))
    s = solver(n, smoother="fused", init_tol=0.0, init_max_cycles=3)
    u = dev(P.initial_guess(p))
    assert s.poisson_init(u, dev(p.f)) == 3
    assert np.abs(host(u) - want).max() <= TOL * np.abs(want).max()


@pytest.mark.parametrize("n,kind", [(64, "exp_cos"), (96, "example4"), (128, "quadratic")])
def test_vcycle_parity_default_smoother(n, kind):
    note("vcycle auto", n, kind)
    p = P.make(kind, n, seed=11)
    u0 = P.initial_guess(p)
    oracle.poisson_init(u0, p.f, oracle.params())
    want = u0.copy()
    for _ in range(2):
        oracle.vcycle(want, p.f, oracle.params())
    s = solver(n)
    u, f = dev(u0), dev(p.f)
    for _ in range(2):
        s.vcycle(u, f)
    assert np.abs(host(u) - want).max() <= TOL * np.abs(want).max()


def test_block_nonconvex_count():
    """A non-convex update is counted once, by the block that owns the node,
    however many neighbouring blocks recompute it in their halos."""
    note("block nonconvex")
    n = 40
    p = P.example4(n)
    f = p.f.copy()
    f[8:10, 8:10, 8:10] = -1.0     # 8 nodes on a block corner of every shape
    u0 = start(p, 3)
    for cfg in (1, 4, 5):
        s = solver(n, smoother="fused", tile_config=cfg)
        nc = s.sweep(dev(u0), dev(f), 2)
        assert nc == 16            # 8 nodes, each updated once per sweep


def _solve(n, kind, seed, init="poisson", **kw):
    p = P.make(kind, n, seed)
    s = solver(n, **kw)
    u = dev(P.initial_guess(p))
    rep = s.solve(u, dev(p.f), tol=1e-9, init=init)
    return host(u), rep


@pytest.mark.parametrize("n,kind,init", [(128, "quadratic", "poisson"), (112, "exp_cos", "poisson"),
                                         (96, "example4", "fmg"), (72, "exp_cos", "poisson")])
def test_solve_bitwise_block_levels_vs_color(n, kind, init):
    """Default policy (block sweeps on the levels with 16 < n <= 64), block
    sweeps everywhere and colour phases everywhere give the same bits and
    the same cycle counts."""
    note("solve block vs color", n, kind, init)
    uc, rc = _solve(n, kind, 5, init, smoother="color")
    ua, ra = _solve(n, kind, 5, init)
    uf, rf = _solve(n, kind, 5, init, smoother="fused")
    assert rc["cycles"] == ra["cycles"] == rf["cycles"]
    assert np.array_equal(ua, uc)
    assert np.array_equal(uf, uc)
    assert ra["nonconvex"] == rc["nonconvex"]


@pytest.mark.parametrize("block_n", [-1, 32, 128])
def test_retune_block_n_same_bits(block_n):
    n = 128
    note("retune block_n", block_n)
    p = P.make("exp_cos", n, 3)
    f = dev(p.f)
    ref = dev(P.initial_guess(p))
    s0 = solver(n)
    r0 = s0.solve(ref, f, tol=1e-8)
    s = solver(n)
    s.retune(block_n=block_n)
    u = dev(P.initial_guess(p))
    r = s.solve(u, f, tol=1e-8)
    assert r["cycles"] == r0["cycles"]
    assert np.array_equal(host(u), host(ref))


def test_batch_mixed_sizes_block_vs_color():
    """A batch whose solves have different sizes at the same depth: the
    depth's block-sweep lists hold every grid, and each solve's result is
    the same as with colour phases."""
    from paper_1411_7018_amd.batch import solve_batch
    specs = [("quadratic", 128, 1), ("exp_cos", 64, 2), ("example4", 96, 3), ("exp_cos", 48, 4)]
    note("batch block vs color")
    res = {}
    for sm in ("color", "auto"):
        solvers, us, fs = [], [], []
        for kind, n, seed in specs:
            p = P.make(kind, n, seed)
            solvers.append(solver(n, smoother=sm))
            us.append(dev(P.initial_guess(p)))
            fs.append(dev(p.f))
        st, reps = solve_batch(solvers, us, fs, tol=1e-9)
        assert st == 0
        res[sm] = ([host(u) for u in us], [r["cycles"] for r in reps])
    assert res["auto"][1] == res["color"][1]
    for a, c in zip(res["auto"][0], res["color"][0]):
        assert np.array_equal(a, c)
