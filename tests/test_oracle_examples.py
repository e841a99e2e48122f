"""Examples 5-7 of Section 4 in the oracle, pinned by Tables 5-7: the
standalone lexicographic Gauss-Seidel solver reproduces the printed
iteration counts, relative residuals and errors; the converged discrete
solutions show the printed orders of accuracy (2 for the smooth Example 5,
about 1.5 for the singular Example 6, about 0.5 or less for Example 7 with
its unbounded gradient)."""
import math

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P


def _gs(p):
    u = P.initial_guess(p, 1.01 * p.u_exact)
    r0 = math.sqrt(oracle.residual(u, p.f, out=False)[1])
    it = 0
    while True:
        oracle.sweep(u, p.f, "lex")
        it += 1
        r = math.sqrt(oracle.residual(u, p.f, out=False)[1])
        if r <= 1e-6 * r0:
            return it, r / r0, np.abs(u - p.u_exact).max()


@pytest.mark.parametrize("kind", ["example5", "example6", "example7"])
@pytest.mark.parametrize("N", [8, 16])
def test_tables5to7_gauss_seidel(golden, kind, N):
    row = {r["N"]: r for r in golden("tables5to7.json")["gauss_seidel"][kind]}[N]
    it, rr, err = _gs(P.make(kind, N))
    assert it == row["iter"]
    assert float(f"{rr:.1e}") == row["relres"]
    assert float(f"{err:.1e}") == row["error"]


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["example5", "example6", "example7"])
def test_tables5to7_gauss_seidel_n32(golden, kind):
    """At N = 32 a sweep lowers the residual by under 1% (Examples 6, 7), so
    the sweep that crosses the tolerance moves with rounding-level changes
    of r^0: the count is pinned to 0.5% (954, 924, 851 against the printed
    954, 925, 854), the error to its printed digits."""
    row = {r["N"]: r for r in golden("tables5to7.json")["gauss_seidel"][kind]}[32]
    it, rr, err = _gs(P.make(kind, 32))
    assert abs(it - row["iter"]) <= 0.005 * row["iter"]
    assert float(f"{err:.1e}") == row["error"]


def test_example5_restated_on_unit_cube():
    """The (0, pi)^3 problem restated on the unit cube: its data satisfy
    det(Hess u) = f with the pi^6 scaling (the exact Hessian of u(pi xi) is
    pi^2 diag(1 + sin))."""
    p = P.example5(8)
    x, y, z = P.grid(8)
    H = [math.pi ** 2 * (1 + np.sin(math.pi * t)) for t in (x, y, z)]
    assert np.allclose(H[0] * H[1] * H[2], p.f, rtol=1e-13)


@pytest.mark.parametrize("kind,lo,hi", [("example5", 1.85, 2.1), ("example6", 1.35, 1.6),
                                        ("example7", 0.1, 0.6)])
def test_orders_of_accuracy(golden, kind, lo, hi):
    """Order between N = 16 and 32 of the converged discrete solution
    (measured 1.93, 1.47, 0.32; Tables 5-7 print 2.0, 1.5 and 0.3 for the
    Gauss-Seidel column)."""
    errs = []
    for N in (16, 32):
        p = P.make(kind, N)
        u = P.initial_guess(p)
        st, rep, _ = oracle.solve_limit(u, p.f)
        assert st == 0
        errs.append(np.abs(u - p.u_exact).max())
    order = math.log2(errs[0] / errs[1])
    assert lo <= order <= hi


@pytest.mark.parametrize("kind", ["example5", "example6", "example7"])
def test_fmg_protocol_iterations(golden, kind):
    """Section 4 protocol (lexicographic, tolerance 1e-6): one FMG-FAS
    iteration is enough from N = 16 on, as printed."""
    rows = {r["N"]: r for r in golden("tables5to7.json")["fmg"][kind]}
    for N in (16, 32):
        p = P.make(kind, N)
        u = P.initial_guess(p)
        st, rep, _ = oracle.solve(u, p.f, oracle.params(order="lex", init="fmg", tol=1e-6))
        assert st == 0 and rep.cycles == rows[N]["iter"] == 1
