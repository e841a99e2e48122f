"""Parity of the HIP FP64 path (through the C ABI) with the CPU oracle.

Each kernel is checked element by element on seeded inputs against the
oracle function for the same step; whole V-cycles and solves are compared
after the same number of cycles (the bar: <= 1e-12 relative max-norm)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu

# FP64 parity bar: <= 1e-12 relative max-norm against the oracle.  The two
# sides use different root methods (closed form vs monotone Newton) and the
# GPU contracts multiply-adds, so agreement is at round-off, not bitwise.
TOL = 1e-12

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


def perturbed(p, amp=0.01, seed=0):
    rng = np.random.default_rng(seed)
    return P.initial_guess(p, p.u_exact * (1.0 + amp * rng.standard_normal(p.u_exact.shape)))


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_7018_amd import Solver  # noqa: F401  loads libmafas.so


def solver(n, **kw):
    from paper_1411_7018_amd import Solver
    return Solver(n, **kw)


@pytest.mark.parametrize("order", ["4c", "8c"])
@pytest.mark.parametrize("n", [2, 3, 8, 17, 40, 67])
def test_sweep_parity(n, order):
    note("sweep", n, order)
    p = P.exp_cos(n, seed=n)
    u0 = perturbed(p, seed=1)
    want = u0.copy()
    oracle.sweep(want, p.f, order)
    oracle.sweep(want, p.f, order)
    s = solver(n, order=order, smoother="color")
    u = dev(u0)
    nc = s.sweep(u, dev(p.f), 2)
    got = host(u)
    assert nc == 0
    assert relmax(got, want) <= TOL
    # Dirichlet layer untouched
    inner = np.zeros_like(got, bool)
    inner[1:-1, 1:-1, 1:-1] = True
    assert np.array_equal(got[~inner], u0[~inner])


@pytest.mark.parametrize("n", [4, 16, 33, 70])
def test_residual_parity(n):
    note("residual", n)
    p = P.example4(n)
    u0 = perturbed(p, seed=2)
    r_want, ss = oracle.residual(u0, p.f)
    s = solver(n)
    r = torch.full_like(dev(u0), 7.0)
    l2 = s.residual(dev(u0), dev(p.f), out=r)
    got = host(r)
    scale = max(np.abs(r_want).max(), np.abs(p.f).max())
    assert np.abs(got - r_want).max() <= TOL * scale
    assert l2 == pytest.approx(oracle.l2(ss, n), rel=1e-12)


@pytest.mark.parametrize("n", [4, 16, 34, 64])
def test_restrict_parity(n):
    note("restrict", n)
    p = P.exp_cos(n, seed=3)
    u0 = perturbed(p, seed=3)
    r, _ = oracle.residual(u0, p.f)
    w_want, b_want = oracle.restrict(u0, r, "ma", oracle.RESTRICT_FULL)
    s = solver(n)
    w, b = s.restrict(dev(u0), dev(p.f))
    assert np.array_equal(host(w), w_want)
    assert np.abs(host(b) - b_want).max() <= TOL * np.abs(b_want).max()


@pytest.mark.parametrize("n", [4, 16, 34, 64])
def test_restrict_half_weighting_parity(n):
    note("restrict-half", n)
    p = P.example4(n)
    u0 = perturbed(p, seed=4)
    r, _ = oracle.residual(u0, p.f)
    w_want, b_want = oracle.restrict(u0, r, "ma", oracle.RESTRICT_HALF)
    s = solver(n, restriction="half")
    w, b = s.restrict(dev(u0), dev(p.f))
    assert np.abs(host(b) - b_want).max() <= TOL * np.abs(b_want).max()


@pytest.mark.parametrize("n", [4, 10, 36, 64])
def test_prolong_parity(n):
    note("prolong", n)
    rng = np.random.default_rng(n)
    nc = n // 2
    uf = rng.standard_normal((n + 1,) * 3)
    uc = rng.standard_normal((nc + 1,) * 3)
    wc = uc.copy()
    wc[1:-1, 1:-1, 1:-1] = rng.standard_normal((nc - 1,) * 3)
    want = uf.copy()
    oracle.prolong_correct(want, uc, wc)
    s = solver(n)
    u = dev(uf)
    s.prolong_correct(u, dev(uc), dev(wc))
    assert np.abs(host(u) - want).max() <= 1e-14


@pytest.mark.parametrize("n", [8, 24, 48])
def test_poisson_init_parity(n):
    note("poisson-init", n)
    p = P.example4(n)
    pr = oracle.params(init_tol=0.0, init_max_cycles=3)
    want = P.initial_guess(p)
    oracle.poisson_init(want, p.f, pr)
    s = solver(n, init_tol=0.0, init_max_cycles=3)
    u = dev(P.initial_guess(p))
    c = s.poisson_init(u, dev(p.f))
    assert c == 3
    assert relmax(host(u), want) <= TOL


@pytest.mark.parametrize("n,kind", [(8, "example4"), (16, "exp_cos"), (24, "quadratic"),
                                    (6, "exp_cos"), (33, "example4")])
def test_vcycle_parity(n, kind):
    note("vcycle", n, kind)
    p = P.make(kind, n, seed=5)
    u0 = P.initial_guess(p)
    oracle.poisson_init(u0, p.f, oracle.params())
    want = u0.copy()
    for _ in range(3):
        oracle.vcycle(want, p.f, oracle.params())
    s = solver(n, smoother="color")
    u = dev(u0)
    f = dev(p.f)
    for _ in range(3):
        s.vcycle(u, f)
    assert relmax(host(u), want) <= TOL


def test_solve_config1_example4_17cubed():
    """17^3 Example 4, Poisson initial guess, V(2,2), tol 1e-10: same cycle
    count and <= 1e-12 relative max-norm agreement with the oracle."""
    note("solve config1")
    n = 16
    p = P.example4(n)
    want = P.initial_guess(p)
    st, rep_o, hist_o = oracle.solve(want, p.f, oracle.params(tol=1e-10))
    assert st == 0
    s = solver(n)
    u = dev(P.initial_guess(p))
    rep = s.solve(u, dev(p.f), tol=1e-10)
    got = host(u)
    assert rep["converged"] == 1
    assert rep["cycles"] == rep_o.cycles
    assert rep["init_cycles"] == rep_o.init_cycles
    assert rep["res0"] == pytest.approx(rep_o.res0, rel=1e-10)
    assert relmax(got, want) <= TOL
    assert np.abs(got - p.u_exact).max() == pytest.approx(2.98e-4, rel=0.01)


@pytest.mark.parametrize("n,kind", [(2, "example4"), (3, "exp_cos"), (5, "quadratic"),
                                    (12, "exp_cos"), (48, "exp_cos")])
def test_solve_parity_edge_sizes(n, kind):
    """Degenerate hierarchies: n=2 (one unknown), odd n (GS only), n=12
    (coarsest n=3)."""
    note("solve edge", n, kind)
    p = P.make(kind, n, seed=7)
    want = P.initial_guess(p)
    st, rep_o, _ = oracle.solve(want, p.f, oracle.params(tol=1e-9, max_cycles=400))
    s = solver(n, max_cycles=400)
    u = dev(P.initial_guess(p))
    rep = s.solve(u, dev(p.f), tol=1e-9)
    assert rep["cycles"] == rep_o.cycles
    assert relmax(host(u), want) <= TOL


def test_config2_quadratic_129_parity_and_exactness():
    """129^3 seeded quadratic (the benchmark workload): two V-cycles match
    the oracle's two V-cycles from the same u0, and the full solve lands on
    the exact quadratic to round-off."""
    note("config2 129^3")
    n = 128
    p = P.quadratic(n, seed=1001)
    u0 = P.initial_guess(p)
    oracle.poisson_init(u0, p.f, oracle.params())
    want = u0.copy()
    for _ in range(2):
        oracle.vcycle(want, p.f, oracle.params())
    s = solver(n)
    u = dev(u0)
    f = dev(p.f)
    for _ in range(2):
        s.vcycle(u, f)
    assert relmax(host(u), want) <= TOL
    u = dev(P.initial_guess(p))
    rep = s.solve(u, f, tol=1e-8)
    assert rep["converged"] == 1
    assert relmax(host(u), p.u_exact) <= 1e-9
    for _ in range(8):                      # continue to the round-off floor
        s.vcycle(u, f)
    assert relmax(host(u), p.u_exact) <= TOL


def test_nonfinite_and_not_converged():
    from paper_1411_7018_amd._lib import MAError, MA_ERR_NONFINITE, MA_ERR_NOT_CONVERGED
    note("errors")
    n = 8
    p = P.example4(n)
    f = p.f.copy()
    f[4, 4, 4] = np.nan
    s = solver(n)
    with pytest.raises(MAError) as ei:
        s.solve(dev(P.initial_guess(p)), dev(f), init_poisson=False)
    assert ei.value.status == MA_ERR_NONFINITE
    s2 = solver(n, max_cycles=1)
    with pytest.raises(MAError) as ei:
        s2.solve(dev(P.initial_guess(p)), dev(p.f), tol=1e-14)
    assert ei.value.status == MA_ERR_NOT_CONVERGED
    assert ei.value.report["cycles"] == 1


def test_nonpositive_f_counted_as_nonconvex():
    note("nonconvex")
    n = 8
    p = P.example4(n)
    f = p.f.copy()
    f[3:5, 3:5, 3:5] = -1.0
    u0 = perturbed(p, seed=9)
    want = u0.copy()
    nc_o = oracle.sweep(want, f, "4c")
    s = solver(n, smoother="color")
    u = dev(u0)
    nc = s.sweep(u, dev(f), 1)
    assert nc == nc_o == 8
    assert relmax(host(u), want) <= TOL


def test_stagnation_above_tolerance_stops_early_like_oracle():
    """Start within round-off of a quadratic's solution, tolerance under the
    FP64 floor: the GPU solve stops not converged once the residual stalls,
    as the oracle does, with a solution at round-off."""
    from paper_1411_7018_amd import Solver, _lib as L
    n = 32
    p = P.quadratic(n, seed=77)
    x, y, z = P.grid(n)
    u0 = p.u_exact + 1e-9 * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    want = u0.copy()
    ost, orep, _ = oracle.solve(want, p.f, oracle.params(tol=1e-12, max_cycles=60, init=False))
    assert ost == 1
    u = torch.from_numpy(u0).cuda()
    with pytest.raises(L.MAError) as ei:
        Solver(n, max_cycles=60).solve(u, torch.from_numpy(p.f).cuda(), tol=1e-12, init="none")
    assert ei.value.status == L.MA_ERR_NOT_CONVERGED
    rep = ei.value.report
    assert 4 <= rep["cycles"] <= 15 and rep["converged"] == 0
    torch.cuda.synchronize()
    assert np.abs(u.cpu().numpy() - p.u_exact).max() <= 1e-13 * np.abs(p.u_exact).max()
