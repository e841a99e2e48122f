"""Pins for the oracle's whole solver: closed-form solutions, printed values
of the paper (Table 3, Figure 1), theorems as invariants, brute force."""
import math

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P


def _spd_everywhere(u):
    n = u.shape[0] - 1
    worst = np.inf
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                g = oracle.hessian(u, i, j, k)
                G = np.array([[g[0], g[3], g[4]], [g[3], g[1], g[5]], [g[4], g[5], g[2]]])
                worst = min(worst, np.linalg.eigvalsh(G)[0])
    return worst


@pytest.mark.parametrize("order", ["4c", "8c", "lex"])
def test_quadratic_reproduced_to_roundoff(order):
    """P1: centred differences are exact for quadratics, so the discrete
    solution is u itself; the solver must land on it."""
    p = P.quadratic(16, seed=21)
    u = P.initial_guess(p)
    st, rep, hist = oracle.solve(u, p.f, oracle.params(order=order, tol=1e-11, max_cycles=60))
    assert st == 0
    assert np.abs(u - p.u_exact).max() <= 1e-12 * np.abs(p.u_exact).max()
    assert rep.nonconvex == 0


def test_quadratic_is_fixed_point_of_local_update():
    p = P.quadratic(8, seed=5)
    u = p.u_exact.copy()
    oracle.sweep(u, p.f, "4c")
    np.testing.assert_allclose(u, p.u_exact, rtol=0, atol=1e-13)


def test_example4_second_order_and_table3(golden):
    """P2: the converged discrete solution of Example 4 decays at second
    order and matches Table 3 (N=8 error 1.2e-3; the Gauss-Seidel column's
    3.0e-4 at N=16, reached at relative residual 1e-6)."""
    errs = {}
    for n in (8, 16, 32):
        p = P.example4(n)
        u = P.initial_guess(p)
        st, rep, _ = oracle.solve(u, p.f, oracle.params(tol=1e-11))
        assert st == 0
        errs[n] = np.abs(u - p.u_exact).max()
    fmg = {r["N"]: r["error"] for r in golden("table3_fmg_error.json")["rows"]}
    gs = {r["N"]: r["error"] for r in golden("table3_gauss_seidel.json")["rows"]}
    assert float(f"{errs[8]:.1e}") == fmg[8]
    assert float(f"{errs[16]:.1e}") == gs[16]
    for a, b in ((8, 16), (16, 32)):
        assert math.log2(errs[a] / errs[b]) == pytest.approx(2.0, abs=0.1)


def test_example4_result_is_convex():
    """P3 / Theorem 2.2: every interior discrete Hessian of the result is SPD."""
    p = P.example4(12)
    u = P.initial_guess(p)
    oracle.solve(u, p.f, oracle.params(tol=1e-12))
    assert _spd_everywhere(u) > 0.5


def test_table3_standalone_gauss_seidel(golden):
    """P14: the lexicographic nonlinear GS solver from 1.01 u reproduces the
    printed iteration counts, residuals and errors of Table 3."""
    for row in golden("table3_gauss_seidel.json")["rows"]:
        n = row["N"]
        if n > 16:
            continue                     # N=32 runs in the slow test below
        p = P.example4(n)
        u = P.initial_guess(p, 1.01 * p.u_exact)
        r0 = math.sqrt(oracle.residual(u, p.f, out=False)[1])
        it = 0
        while True:
            oracle.sweep(u, p.f, "lex")
            it += 1
            r = math.sqrt(oracle.residual(u, p.f, out=False)[1])
            if r <= 1e-6 * r0:
                break
        assert it == row["iter"]
        assert float(f"{r / r0:.1e}") == row["relres"]
        assert float(f"{np.abs(u - p.u_exact).max():.1e}") == row["error"]


@pytest.mark.slow
def test_table3_standalone_gauss_seidel_n32(golden):
    row = [r for r in golden("table3_gauss_seidel.json")["rows"] if r["N"] == 32][0]
    p = P.example4(32)
    u = P.initial_guess(p, 1.01 * p.u_exact)
    r0 = math.sqrt(oracle.residual(u, p.f, out=False)[1])
    it = 0
    while True:
        oracle.sweep(u, p.f, "lex")
        it += 1
        r = math.sqrt(oracle.residual(u, p.f, out=False)[1])
        if r <= 1e-6 * r0:
            break
    assert it == row["iter"]
    assert float(f"{np.abs(u - p.u_exact).max():.1e}") == row["error"]
    assert r / r0 == pytest.approx(row["relres"], rel=0.07)


def test_figure1_smoothing(golden):
    """P13: Figure 1's maxima 1.4712 -> 0.7538 after two lexicographic
    sweeps, reproduced on h = 1/32 with the Example 4 data."""
    g = golden("figure1.json")
    n = g["N"]
    p = P.example4(n)
    u = P.initial_guess(p, p.u_exact + P.figure1_error(n))
    assert round(np.abs(u - p.u_exact).max(), 4) == g["max_error_before"]
    oracle.sweep(u, p.f, "lex")
    oracle.sweep(u, p.f, "lex")
    assert round(np.abs(u - p.u_exact).max(), 4) == g["max_error_after_two_sweeps"]


def _ma_system(u_int, n, f, g_full):
    u = g_full.copy()
    u[1:-1, 1:-1, 1:-1] = u_int.reshape((n - 1,) * 3)
    s = float(n * n)
    c = u[1:-1, 1:-1, 1:-1]
    sl = lambda dk, dj, di: u[1 + dk:n + dk, 1 + dj:n + dj, 1 + di:n + di]   # noqa: E731
    xx = (sl(0, 0, 1) + sl(0, 0, -1) - 2 * c) * s
    yy = (sl(0, 1, 0) + sl(0, -1, 0) - 2 * c) * s
    zz = (sl(1, 0, 0) + sl(-1, 0, 0) - 2 * c) * s
    xy = (sl(0, 1, 1) + sl(0, -1, -1) - sl(0, 1, -1) - sl(0, -1, 1)) * s / 4
    xz = (sl(1, 0, 1) + sl(-1, 0, -1) - sl(1, 0, -1) - sl(-1, 0, 1)) * s / 4
    yz = (sl(1, 1, 0) + sl(-1, -1, 0) - sl(1, -1, 0) - sl(-1, 1, 0)) * s / 4
    det = xx * yy * zz + 2 * xy * yz * xz - xx * yz ** 2 - yy * xz ** 2 - zz * xy ** 2
    return (det - f[1:-1, 1:-1, 1:-1]).ravel()


def _newton_fd(x0, fun, iters=30):
    """Plain Newton on the 27 equations with a central-difference Jacobian."""
    x = x0.copy()
    for _ in range(iters):
        F0 = fun(x)
        J = np.empty((x.size, x.size))
        for m in range(x.size):
            e = np.zeros_like(x)
            e[m] = 1e-6 * max(1.0, abs(x[m]))
            J[:, m] = (fun(x + e) - fun(x - e)) / (2 * e[m])
        dx = np.linalg.solve(J, -F0)
        x = x + dx
        if np.abs(dx).max() <= 1e-15 * np.abs(x).max():
            break
    return x


@pytest.mark.parametrize("kind", ["example4", "exp_cos"])
def test_brute_force_5cubed(kind):
    """P4: on the 5^3 grid (27 unknowns) plain Newton on the 27 discrete
    equations (finite-difference Jacobian), started from several perturbed
    convex guesses, lands on the point the V-cycle converges to (<= 1e-12),
    and scipy's fsolve agrees from the exact solution."""
    from scipy.optimize import fsolve
    n = 4
    p = P.make(kind, n, seed=9)
    u = P.initial_guess(p)
    st, rep, _ = oracle.solve_limit(u, p.f)
    fun = lambda x: _ma_system(x, n, p.f, p.u_exact)   # noqa: E731
    rng = np.random.default_rng(1)
    want = u[1:-1, 1:-1, 1:-1].ravel()
    for trial in range(3):
        x0 = (p.u_exact[1:-1, 1:-1, 1:-1] * (1 + 0.01 * rng.standard_normal((3, 3, 3)))).ravel()
        sol = _newton_fd(x0, fun)
        assert np.abs(fun(sol)).max() <= 1e-9 * np.abs(p.f).max()
        assert np.abs(sol - want).max() <= 1e-12
    sol = fsolve(fun, p.u_exact[1:-1, 1:-1, 1:-1].ravel(), xtol=1e-14)
    assert np.abs(sol - want).max() <= 1e-10
    assert _spd_everywhere(u) > 0


@pytest.mark.parametrize("n", [16, 32])
def test_poisson_vcycle_contraction(n):
    """P12: linear V(2,2) on the 7-point Laplacian with 4-colour GS and full
    weighting contracts by <= 0.15 per cycle, independently of n."""
    p = P.example4(n)
    u = P.initial_guess(p)
    R = oracle.poisson_rhs(p.f)
    pr = oracle.params()
    r = [math.sqrt(oracle.poisson_residual(u, R)[1])]
    for _ in range(6):
        oracle.poisson_vcycle(u, R, pr)
        r.append(math.sqrt(oracle.poisson_residual(u, R)[1]))
    rates = np.array(r[1:]) / np.array(r[:-1])
    assert rates.max() <= 0.15


def test_half_weighting_with_colours_diverges_full_weighting_does_not():
    """Why colour orderings use full weighting: with half-weighting the
    4-colour linear V-cycle loses its contraction as n grows."""
    def rate(rmode, n):
        p = P.example4(n)
        u = P.initial_guess(p)
        R = oracle.poisson_rhs(p.f)
        pr = oracle.params(rmode=rmode)
        r = []
        for _ in range(8):
            oracle.poisson_vcycle(u, R, pr)
            r.append(math.sqrt(oracle.poisson_residual(u, R)[1]))
        return r[-1] / r[-2]
    assert rate(oracle.RESTRICT_HALF, 32) > 0.5
    assert rate(oracle.RESTRICT_FULL, 32) < 0.15


def test_ma_vcycle_mesh_independent_rate():
    """The 4-colour FAS V(2,2) with full weighting contracts the MA residual
    at a rate that does not grow with n (measured over the first cycles)."""
    rates = {}
    for n in (16, 32):
        p = P.exp_cos(n, seed=2)
        u = P.initial_guess(p)
        st, rep, hist = oracle.solve(u, p.f, oracle.params(tol=1e-8))
        assert st == 0
        rates[n] = (hist[4] / hist[0]) ** 0.25
    assert rates[32] < 0.2 and rates[16] < 0.2


def test_fixed_point_of_vcycle_tau_consistency():
    """P10: one V-cycle from the converged discrete solution changes nothing
    beyond round-off (FAS tau-correction consistency)."""
    p = P.exp_cos(16, seed=4)
    u = P.initial_guess(p)
    oracle.solve_limit(u, p.f)
    v = u.copy()
    oracle.vcycle(v, p.f)
    assert np.abs(v - u).max() <= 1e-13


def test_levels():
    assert oracle.levels(16) == [16, 8, 4, 2]
    assert oracle.levels(96) == [96, 48, 24, 12, 6, 3]
    assert oracle.levels(384) == [384, 192, 96, 48, 24, 12, 6, 3]
    assert oracle.levels(2) == [2]
    assert oracle.levels(7) == [7]


def test_odd_coarsest_level_converges():
    """n = 24 ends on a 4^3 grid (n_L = 3, 8 unknowns) with one sweep there."""
    p = P.exp_cos(24, seed=8)
    u = P.initial_guess(p)
    st, rep, hist = oracle.solve(u, p.f, oracle.params(tol=1e-9))
    assert st == 0 and rep.cycles <= 20


def test_limit_mode_reaches_roundoff_floor():
    p = P.example4(16)
    u = P.initial_guess(p)
    st, rep, hist = oracle.solve_limit(u, p.f)
    assert st == 0
    assert rep.res / rep.res0 < 1e-12


def test_stagnation_above_tolerance_stops_early():
    """A start within round-off of a quadratic's exact discrete solution: the
    relative tolerance lies under the FP64 floor, the residual stalls (three
    cycles in a row without dropping below 0.9 x its best) and the solve
    stops not converged, long before max_cycles."""
    p = P.quadratic(32, seed=77)
    x, y, z = P.grid(32)
    bump = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    u = p.u_exact + 1e-9 * bump
    st, rep, hist = oracle.solve(u, p.f, oracle.params(tol=1e-12, max_cycles=60, init=False))
    assert st == 1 and rep.converged == 0
    assert 4 <= rep.cycles <= 15
    assert rep.res > 1e-12 * rep.res0
    # it did reach the floor: the solution is the quadratic to round-off
    assert np.abs(u - p.u_exact).max() <= 1e-13 * np.abs(p.u_exact).max()
