"""The fused 4-colour sweep (one launch per sweep, LDS ring, skewed phases)
against the per-colour kernel (bitwise: same point-update code on the same
neighbour values) and against the oracle (<= 1e-12 relative)."""
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


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("n,zc", [(32, 0), (47, 5), (70, 1), (100, 0)])
def test_fused_sweep_bitwise_vs_color_and_oracle(n, zc, cfg):
    note("fused sweep", n, zc, cfg)
    p = P.exp_cos(n, seed=n + cfg)
    u0 = start(p, cfg)
    f = dev(p.f)
    uc = dev(u0)
    solver(n, smoother="color").sweep(uc, f, 2)
    uf = dev(u0)
    solver(n, smoother="fused", tile_config=cfg, zchunk=zc).sweep(uf, f, 2)
    got, ref = host(uf), host(uc)
    assert np.array_equal(got, ref)
    want = u0.copy()
    oracle.sweep(want, p.f, "4c")
    oracle.sweep(want, p.f, "4c")
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()


@pytest.mark.parametrize("n", [40, 64])
def test_fused_poisson_init_parity(n):
    note("fused poisson", n)
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


def test_fused_nonconvex_count():
    note("fused nonconvex")
    n = 40
    p = P.example4(n)
    f = p.f.copy()
    f[10:12, 10:12, 10:12] = -1.0
    u0 = start(p, 3)
    s = solver(n, smoother="fused", tile_config=3, zchunk=4)
    nc = s.sweep(dev(u0), dev(f), 2)
    assert nc == 16        # 8 nodes, each updated once per sweep
