"""Pins for the oracle's Poisson initial guess (the linear problem
Lap_h u0 = 3 f^(1/3) with the Dirichlet data of u, solved by linear V(2,2)
cycles with the colour ordering and transfers of the FAS cycle).

Each pin is fixed by mathematics outside the oracle:
  * the 7-point centred Laplacian is exact on polynomials of degree <= 3 in
    each variable, so on such a u the discrete residual is R - Lap u with
    Lap u written out by hand;
  * on a quadratic u = x^T A x / 2 + b^T x, Lap u = tr A, and with
    f = (tr A / 3)^3 the Poisson right-hand side 3 f^(1/3) is tr A, so the
    discrete Poisson problem has u itself as its solution;
  * 3 f^(1/3) at perfect cubes is a known number.
A wrong scale or sign of the Laplacian, a wrong root, or a wrong update
rule breaks at least one of them."""
import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P


def _quadratic_fields(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    A = Q @ np.diag(rng.uniform(0.5, 2.0, 3)) @ Q.T
    b = rng.uniform(-1.0, 1.0, 3)
    X, Y, Z = P.grid(n)
    pts = np.stack([X, Y, Z], axis=-1)
    u = 0.5 * np.einsum("...a,ab,...b->...", pts, A, pts) + pts @ b
    return u, A


@pytest.mark.parametrize("f,want", [(8.0, 6.0), (27.0, 9.0), (1.0, 3.0), (0.0, 0.0),
                                    (0.125, 1.5), (1000.0, 30.0)])
def test_poisson_rhs_is_three_cube_roots(f, want):
    """3 f^(1/3) at perfect cubes, to the rounding of the library cube root
    (glibc's cbrt is within an ulp, not correctly rounded)."""
    R = oracle.poisson_rhs(np.full((3, 3, 3), f))
    assert np.abs(R - want).max() <= 4 * np.finfo(float).eps * want


@pytest.mark.parametrize("n", [8, 16])
def test_poisson_residual_of_quadratic_is_R_minus_trace(n):
    """Lap_h of a quadratic is tr A at every interior node (exactly, up to
    rounding), and the residual is 0 on the Dirichlet layer."""
    u, A = _quadratic_fields(n, 7 + n)
    R = np.random.default_rng(3).uniform(-2.0, 2.0, u.shape)
    r, ss = oracle.poisson_residual(u, R)
    inner = (slice(1, -1),) * 3
    want = R[inner] - np.trace(A)
    scale = np.abs(u).max() * n * n
    assert np.abs(r[inner] - want).max() <= 64 * np.finfo(float).eps * scale
    assert np.all(r[0] == 0) and np.all(r[-1] == 0)
    assert np.all(r[:, 0] == 0) and np.all(r[:, :, -1] == 0)
    assert ss == pytest.approx(float((r[inner] ** 2).sum()), rel=1e-12)


def test_poisson_residual_of_cubic_is_exact_laplacian():
    """u = x^3 + 2 y^2 z - x y z + z^3 / 3 has u_xx = 6x, u_yy = 4z and
    u_zz = 2z; centred second differences are exact on cubics, so with
    R = 0 the residual is -(6x + 6z) at every interior node."""
    n = 12
    X, Y, Z = P.grid(n)
    u = X ** 3 + 2 * Y ** 2 * Z - X * Y * Z + Z ** 3 / 3
    R = np.zeros_like(u)
    r, _ = oracle.poisson_residual(u, R)
    inner = (slice(1, -1),) * 3
    lap = 6 * X + 6 * Z
    assert np.abs(r[inner] + lap[inner]).max() <= 1e-10


@pytest.mark.parametrize("n,order", [(16, "4c"), (16, "8c"), (12, "lex"), (24, "4c")])
def test_poisson_init_reproduces_quadratic(n, order):
    """With f = (tr A / 3)^3 the Poisson problem's exact solution is the
    quadratic itself; the oracle's Poisson guess must return it from a zero
    interior (any Laplacian scale, sign or root error moves it away)."""
    u_exact, A = _quadratic_fields(n, 100 + n)
    f = np.full_like(u_exact, (np.trace(A) / 3.0) ** 3)
    u = u_exact.copy()
    u[1:-1, 1:-1, 1:-1] = 0.0
    cycles = oracle.poisson_init(u, f, oracle.params(order=order, init_tol=1e-14,
                                                     init_max_cycles=60))
    assert 1 <= cycles <= 60
    assert np.abs(u - u_exact).max() <= 1e-12 * np.abs(u_exact).max()


def test_poisson_init_single_update_closed_form():
    """n = 2: one unknown; one linear update sets it to the mean of its six
    neighbours minus h^2 R / 6 (the 7-point equation solved exactly)."""
    n = 2
    rng = np.random.default_rng(11)
    u = rng.uniform(0.0, 1.0, (3, 3, 3))
    f = np.full((3, 3, 3), 8.0)          # R = 6
    want = (u[1, 1, 0] + u[1, 1, 2] + u[1, 0, 1] + u[1, 2, 1] + u[0, 1, 1] + u[2, 1, 1]) / 6.0 \
        - (0.5 ** 2) * 6.0 / 6.0
    oracle.poisson_init(u, f, oracle.params(init_tol=1e-14, init_max_cycles=1))
    assert u[1, 1, 1] == pytest.approx(want, rel=1e-15, abs=1e-15)
