"""The 2D variant on the GPU (include/ma2d.h) against the 2D oracle: sweeps
in both orderings, residual, V-cycles, FMG and full solves under the
Section 4 protocol, including Table 1's 'Iter' and 'Error'."""
import sys

import numpy as np
import pytest

from oracle import ma2
from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
TOL = 1e-12
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def note(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def perturbed(p, seed=0, amp=0.01):
    rng = np.random.default_rng(seed)
    return P.initial_guess2(p, p.u_exact * (1 + amp * rng.standard_normal(p.u_exact.shape)))


ORD = {"rb": 0, "4c": 1}


@pytest.mark.parametrize("n", [2, 3, 8, 33, 64, 130])
@pytest.mark.parametrize("order", ["rb", "4c"])
def test_sweep_parity(n, order):
    from paper_1411_7018_amd.solver2d import Solver2D
    note("2d sweep", n, order)
    p = P.example2d(1, n)
    u0 = perturbed(p, seed=n)
    want = u0.copy()
    nco = ma2.sweep(want, p.f, order) + ma2.sweep(want, p.f, order)
    u = dev(u0)
    ncg = Solver2D(n, order=order).sweep(u, dev(p.f), 2)
    assert relmax(host(u), want) <= TOL and ncg == nco


@pytest.mark.parametrize("n", [4, 17, 100])
def test_residual_parity(n):
    from paper_1411_7018_amd.solver2d import Solver2D
    p = P.example2d(2, n)
    u0 = perturbed(p, seed=1)
    r_o, ss = ma2.residual(u0, p.f)
    out = dev(np.zeros_like(u0))
    l2 = Solver2D(n).residual(dev(u0), dev(p.f), out)
    scale = max(np.abs(r_o).max(), np.abs(p.f).max())
    assert np.abs(host(out) - r_o).max() <= TOL * scale
    assert l2 == pytest.approx(np.sqrt(ss) / n, rel=1e-12)


@pytest.mark.parametrize("n,order,rm", [(8, "rb", 0), (24, "rb", 0), (64, "4c", 1),
                                        (128, "rb", 0), (96, "4c", 1)])
def test_vcycle_and_fmg_parity(n, order, rm):
    from paper_1411_7018_amd.solver2d import Solver2D
    note("2d vcycle/fmg", n, order, rm)
    p = P.example2d(1, n)
    pr = ma2.params(order=order, rmode=rm)
    s = Solver2D(n, order=order, restriction="half" if rm == 0 else "full")
    want = P.initial_guess2(p)
    ma2.fmg(want, p.f, pr)
    u = dev(P.initial_guess2(p, 0.5))
    s.fmg(u, dev(p.f))
    assert relmax(host(u), want) <= TOL
    for _ in range(2):
        ma2.vcycle(want, p.f, pr)
        s.vcycle(u, dev(p.f))
    assert relmax(host(u), want) <= TOL


@pytest.mark.parametrize("ex", [1, 2, 3])
@pytest.mark.parametrize("N", [128, 256, 512])
def test_table1_solve_on_gpu(golden, ex, N):
    """Red-black, half-weighting, tolerance 1e-6 from the FMG start: the same
    cycle count and result as the oracle, and Table 1's 'Iter' and 'Error'."""
    from paper_1411_7018_amd.solver2d import Solver2D
    note("2d table1", ex, N)
    row = {r["N"]: r for r in golden("tables1_2.json")["red_black"][str(ex)]}[N]
    p = P.example2d(ex, N)
    want = P.initial_guess2(p)
    st, rep_o = ma2.solve(want, p.f, ma2.params(order="rb", rmode=0, tol=1e-6))
    u = dev(P.initial_guess2(p, 0.3))
    rep = Solver2D(N).solve(u, dev(p.f), tol=1e-6)
    assert rep["converged"] == 1 and rep["cycles"] == rep_o.cycles == row["iter"]
    got = host(u)
    assert relmax(got, want) <= TOL
    err = np.abs(got - p.u_exact).max()
    assert abs(err - row["error"]) <= 0.06 * row["error"]


def test_2d_errors():
    from paper_1411_7018_amd import _lib as L
    from paper_1411_7018_amd.solver2d import Solver2D
    p = P.example2d(1, 16)
    s = Solver2D(16, max_cycles=1)
    u = dev(P.initial_guess2(p))
    with pytest.raises(L.MAError) as ei:
        s.solve(u, dev(p.f), tol=1e-30)
    assert ei.value.status == L.MA_ERR_NOT_CONVERGED and ei.value.report["cycles"] == 1
    with pytest.raises(TypeError):
        s.solve(u.float(), dev(p.f))
