"""FP32/FP64 mixed-precision form (outer FP64 defect correction, inner FP32
FAS cycles on the correction).  Its fixed point is the FP64 discrete
solution, so it is checked against the oracle run to its round-off limit and
against the plain FP64 GPU path."""
import sys

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def solve(n, p, precision, tol, **kw):
    from paper_1411_7018_amd import Solver
    s = Solver(n, precision=precision, **kw)
    u = dev(P.initial_guess(p))
    rep = s.solve(u, dev(p.f), tol=tol)
    torch.cuda.synchronize()
    return u.cpu().numpy(), rep


@pytest.mark.parametrize("n,kind", [(16, "example4"), (32, "exp_cos"), (48, "exp_cos"),
                                    (64, "exp_cos"), (24, "quadratic")])
def test_mixed_matches_oracle_limit(n, kind):
    """Both forms, run to 1e-10 relative residual, agree with the oracle's
    converged discrete solution to <= 1e-10 in the max norm."""
    note("mixed vs oracle limit", n, kind)
    p = P.make(kind, n, seed=3001)
    lim = P.initial_guess(p)
    oracle.solve_limit(lim, p.f)
    um, rm = solve(n, p, "mixed", 1e-10)
    ud, rd = solve(n, p, "fp64", 1e-10)
    assert rm["converged"] == 1 and rd["converged"] == 1
    assert rm["outer"] >= 1
    assert np.abs(um - lim).max() <= 1e-10
    assert np.abs(ud - lim).max() <= 1e-10
    # the inner FP32 cycles converge like the FP64 ones
    assert rm["cycles"] <= rd["cycles"] + 4


def test_config3_mixed_vs_fp64_257():
    """257^3 exp + cosines: mixed and FP64 both reach 1e-8; at 1e-10 they
    agree to <= 1e-10; FP64 fallbacks stay a small fraction of updates."""
    note("config3 257^3")
    n = 256
    p = P.exp_cos(n, seed=3001)
    um8, rm8 = solve(n, p, "mixed", 1e-8)
    ud8, rd8 = solve(n, p, "fp64", 1e-8)
    assert rm8["converged"] == 1 and rd8["converged"] == 1
    assert rm8["rel_res"] <= 1e-8 and rd8["rel_res"] <= 1e-8
    assert rm8["fp64_fallbacks"] <= 1e-2 * rm8["point_updates"]
    um, rm = solve(n, p, "mixed", 1e-10)
    ud, rd = solve(n, p, "fp64", 1e-10)
    assert np.abs(um - ud).max() <= 1e-10
    assert np.abs(um - p.u_exact).max() == pytest.approx(np.abs(ud - p.u_exact).max(), rel=1e-6)


def test_mixed_nonpositive_f_counted():
    """Nodes where F <= 0 leave the certified FP32 branch: they are solved in
    FP64 with the general root rule and counted as non-convex."""
    note("mixed nonconvex")
    n = 16
    p = P.example4(n)
    p.f = p.f.copy()
    p.f[7:9, 7:9, 7:9] = -0.5
    from paper_1411_7018_amd import Solver
    from paper_1411_7018_amd._lib import MAError
    s = Solver(n, precision="mixed", max_cycles=3)
    u = dev(P.initial_guess(p))
    try:
        rep = s.solve(u, dev(p.f), tol=1e-12)
    except MAError as e:
        rep = e.report
    assert rep["nonconvex"] > 0 and rep["fp64_fallbacks"] > 0
    assert np.isfinite(u.cpu().numpy()).all()


def test_mixed_8_colour_order():
    note("mixed 8c")
    n = 32
    p = P.exp_cos(n, seed=7)
    lim = P.initial_guess(p)
    oracle.solve_limit(lim, p.f, order="8c")
    um, rm = solve(n, p, "mixed", 1e-10, order="8c")
    assert rm["converged"] == 1
    assert np.abs(um - lim).max() <= 1e-10
