"""The 2D variant in the oracle (u_xx u_yy - u_xy^2 = f, 9-point stencil),
pinned by what the paper and the mathematics fix: the smaller root of the
local quadratic (against numpy.roots, and the only one leaving the Hessian
positive definite), quadratic solutions reproduced to round-off, the
4-colour ordering decoupling the 9-point stencil (red-black does not), and
Tables 1-2: 'Iter' and 'Error' of FMG-FAS on Examples 1-3."""
import math

import numpy as np
import pytest

from oracle import ma2
from paper_1411_7018_amd import problems as P


def test_local_root_smaller_and_convex():
    rng = np.random.default_rng(3)
    for _ in range(300):
        A = rng.standard_normal((2, 2))
        G = A @ A.T + 0.1 * np.eye(2)
        g = np.array([G[0, 0], G[1, 1], G[0, 1]])
        F = float(rng.uniform(0.01, 3.0))
        sig, nc = ma2.local_root(g, F)
        roots = np.roots([1.0, -(g[0] + g[1]), g[0] * g[1] - g[2] ** 2 - F])
        assert not nc
        assert sig == pytest.approx(min(roots.real), rel=1e-12, abs=1e-12)
        assert np.all(np.linalg.eigvalsh(G - sig * np.eye(2)) > 0)     # convex
        big = max(roots.real)
        assert not np.all(np.linalg.eigvalsh(G - big * np.eye(2)) > 0)


def test_local_root_no_cancellation():
    """d - F tiny against tr: the stable form keeps full relative accuracy."""
    g = np.array([1.0, 1.0, 0.0])
    F = 1.0 - 1e-12                      # exact smaller root ~ 5e-13
    sig, _ = ma2.local_root(g, F)
    exact = (2.0 - math.sqrt(4.0 * F)) / 2.0
    assert sig == pytest.approx(1e-12 / (1.0 + math.sqrt(F)), rel=1e-9)
    assert abs(sig - 5e-13) < 1e-15 or abs(sig - exact) < 1e-15


def test_no_real_root_counts_nonconvex():
    sig, nc = ma2.local_root(np.array([1.0, 1.0, 0.0]), -5.0)
    assert nc and sig == pytest.approx(1.0)


def _quadratic2d(n, seed=0):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((2, 2)))
    A = (q * rng.uniform(0.5, 2.0, 2)) @ q.T
    A = 0.5 * (A + A.T)
    b = rng.uniform(-1, 1, 2)
    x, y = P.grid2(n)
    u = 0.5 * (A[0, 0] * x * x + A[1, 1] * y * y) + A[0, 1] * x * y + b[0] * x + b[1] * y
    return u, np.full_like(u, np.linalg.det(A))


@pytest.mark.parametrize("order,rmode", [("4c", 1), ("rb", 0), ("lex", 0)])
def test_quadratic_reproduced(order, rmode):
    ue, f = _quadratic2d(32)
    u = ue.copy()
    u[1:-1, 1:-1] = 0.0
    st, rep = ma2.solve(u, f, ma2.params(order=order, rmode=rmode, tol=-1.0, max_cycles=80))
    assert st == 0
    assert np.abs(u - ue).max() <= 1e-12


def test_four_colours_decouple_nine_point_stencil():
    offs = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]
    for i in range(4):
        for j in range(4):
            c = (i & 1) + 2 * (j & 1)
            assert all(((i + a) & 1) + 2 * ((j + b) & 1) != c for a, b in offs)
    # red-black leaves the diagonal neighbours in the same colour
    assert ((0 + 0) & 1) == ((1 + 1) & 1)


def _table(golden, order, ex):
    key = "red_black" if order == "rb" else "lexicographic"
    return golden("tables1_2.json")[key][str(ex)]


@pytest.mark.parametrize("ex", [1, 2, 3])
def test_table1_red_black(golden, ex):
    for row in _table(golden, "rb", ex):
        if row["N"] > 512:
            continue
        p = P.example2d(ex, row["N"])
        u = P.initial_guess2(p)
        st, rep = ma2.solve(u, p.f, ma2.params(order="rb", rmode=0, tol=1e-6))
        assert st == 0 and rep.cycles == row["iter"]
        err = np.abs(u - p.u_exact).max()
        assert abs(err - row["error"]) <= 0.06 * row["error"]


@pytest.mark.parametrize("ex", [1, 2])
def test_table2_lexicographic(golden, ex):
    for row in _table(golden, "lex", ex):
        if row["N"] > 512:
            continue
        p = P.example2d(ex, row["N"])
        u = P.initial_guess2(p)
        st, rep = ma2.solve(u, p.f, ma2.params(order="lex", rmode=0, tol=1e-6))
        assert st == 0 and rep.cycles == row["iter"]
        err = np.abs(u - p.u_exact).max()
        assert abs(err - row["error"]) <= 0.08 * row["error"]


@pytest.mark.parametrize("ex,lo,hi", [(1, 1.95, 2.05), (2, 1.45, 1.55), (3, 0.45, 0.55)])
def test_orders_2d(ex, lo, hi):
    errs = []
    for N in (128, 256):
        p = P.example2d(ex, N)
        u = P.initial_guess2(p)
        ma2.solve(u, p.f, ma2.params(order="rb", rmode=0, tol=1e-6))
        errs.append(np.abs(u - p.u_exact).max())
    assert lo <= math.log2(errs[0] / errs[1]) <= hi


def test_fmg2_interp_exact_on_bicubics():
    rng = np.random.default_rng(1)
    C = rng.standard_normal((4, 4))
    def field(n):
        x, y = P.grid2(n)
        return sum(C[a, b] * x ** a * y ** b for a in range(4) for b in range(4))
    uc = field(8)
    uf = np.zeros((17, 17))
    ma2.fmg_interp(uc, uf)
    want = field(16)
    assert np.abs(uf[1:-1, 1:-1] - want[1:-1, 1:-1]).max() <= 1e-12
