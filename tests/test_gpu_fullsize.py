"""Parity at the benchmark's full sizes, where the oracle cannot run whole
solves in test time:

* one GPU sweep (colour launches) at 129^3, 257^3 and 385^3, checked node by
  node on samples of every colour: a colour-c node's new value depends only
  on F, its own old value, the new values of its neighbours of colours < c
  and the old values of those of colours > c, all of which are known from
  the sweep's input and output, so the oracle's pointwise update (its
  Hessian and root rule) recomputes it exactly;
* the residual at full size on sampled nodes;
* the V-cycle in the launch structure the benchmark times (tuned launch
  shape, block sweeps, fused residual-restriction, coarse levels in LDS)
  against the unfused colour-launch form, bitwise, at 257^3;
* the 64-solve batch of the batch workload: sampled members bitwise equal to
  the same problem solved alone.
"""
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


def start(kind, n, seed):
    """Problem data and the Poisson initial guess computed on the GPU."""
    p = P.make(kind, n, seed)
    u = dev(P.initial_guess(p))
    f = dev(p.f)
    solver(n).poisson_init(u, f)
    return p, u, f


def colours(n):
    k, j, i = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    return ((i + j) & 1) + 2 * ((i + k) & 1)


def check_sweep_samples(uin, uout, F, samples=600, seed=0):
    n = uin.shape[0] - 1
    col = colours(n)
    rng = np.random.default_rng(seed)
    half_h2 = 0.5 / (float(n) * float(n))
    scale = np.abs(uout).max()
    worst = 0.0
    for c in range(4):
        mixed = np.where(col < c, uout, uin)
        mixed = np.ascontiguousarray(mixed)
        kk, jj, ii = np.nonzero((col == c)[1:-1, 1:-1, 1:-1])
        pick = rng.choice(len(ii), size=min(samples, len(ii)), replace=False)
        for q in pick:
            i, j, k = int(ii[q]) + 1, int(jj[q]) + 1, int(kk[q]) + 1
            g = oracle.hessian(mixed, i, j, k)
            sig = oracle.local_root(g, float(F[k, j, i]))
            want = mixed[k, j, i] + sig * half_h2
            worst = max(worst, abs(uout[k, j, i] - want))
    assert worst <= TOL * scale, (worst, scale)
    # the Dirichlet layer is untouched
    inner = np.zeros_like(col, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    assert np.array_equal(uout[~inner], uin[~inner])


@pytest.mark.parametrize("kind,n,seed", [("quadratic", 128, 1001), ("exp_cos", 256, 3001),
                                         ("exp_cos", 384, 5001)])
def test_sweep_full_size_sampled(kind, n, seed):
    note("full-size sweep", kind, n)
    p, u, f = start(kind, n, seed)
    uin = host(u)
    solver(n, smoother="color").sweep(u, f, 1)
    check_sweep_samples(uin, host(u), p.f, seed=n)


def test_block_sweep_full_size_equals_colour():
    n = 256
    note("full-size block sweep")
    p, u, f = start("exp_cos", n, 3001)
    ub = u.clone()
    solver(n, smoother="color").sweep(u, f, 2)
    solver(n, smoother="fused").sweep(ub, f, 2)
    assert np.array_equal(host(ub), host(u))


@pytest.mark.parametrize("kind,n,seed", [("exp_cos", 256, 3001), ("exp_cos", 384, 5001)])
def test_residual_full_size_sampled(kind, n, seed):
    note("full-size residual", kind, n)
    p, u, f = start(kind, n, seed)
    r = torch.empty_like(u)
    l2 = solver(n).residual(u, f, r)
    uh, rh = host(u), host(r)
    rng = np.random.default_rng(n)
    scale = np.abs(p.f).max()
    for _ in range(2000):
        i, j, k = (int(x) for x in rng.integers(1, n, size=3))
        want = p.f[k, j, i] - oracle.det3(oracle.hessian(uh, i, j, k))
        assert abs(rh[k, j, i] - want) <= TOL * scale
    h = 1.0 / n
    assert l2 == pytest.approx(np.sqrt(h ** 3 * np.sum(rh.astype(np.float64) ** 2)), rel=1e-12)


def test_vcycle_full_size_bench_structure_equals_unfused():
    n = 256
    note("full-size vcycle")
    p, u, f = start("exp_cos", n, 3001)
    uc = u.clone()
    s = solver(n, coarse_n=16, max_blocks=65536, strip_rows=128)   # a tuned shape
    c = solver(n, smoother="color", coarse_n=0)
    for _ in range(2):
        s.vcycle(u, f)
        c.vcycle(uc, f)
    assert np.array_equal(host(u), host(uc))


def test_batch64_members_equal_solo():
    from paper_1411_7018_amd.batch import solve_batch
    note("full-size batch")
    specs = P.batch_specs(64)
    data = [P.make_device(k, n, sd) for k, n, sd in specs]
    solvers = [solver(n) for _, n, _ in specs]
    us = [d[0].clone() for d in data]
    st, reps = solve_batch(solvers, us, [d[1] for d in data], tol=1e-8)
    assert st == 0 and all(r["converged"] == 1 for r in reps)
    for m in (0, 9, 21, 33, 47, 63):
        kind, n, sd = specs[m]
        u0, f = P.make_device(kind, n, sd)
        rep = solver(n).solve(u0, f, tol=1e-8)
        assert rep["cycles"] == reps[m]["cycles"]
        assert np.array_equal(host(u0), host(us[m])), m
