"""Pins for the oracle's pointwise pieces: discrete Hessian (eqs. 2.1-2.6),
determinant (the explicit operator of Section 1), and the local root rule
(eqs. 2.8-2.9, Theorems 2.1-2.2).  Each check uses an independent route:
numpy eigenvalues / companion-matrix roots, closed forms, or bisection."""
import math

import numpy as np
import pytest

import oracle


def _sym(g):
    xx, yy, zz, xy, xz, yz = g
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def _min_real_root(coeffs):
    r = np.roots(coeffs)
    real = r[np.abs(r.imag) <= 1e-7 * np.maximum(1.0, np.abs(r.real))].real
    return real.min()


def test_det3_matches_linalg():
    rng = np.random.default_rng(1)
    for _ in range(200):
        g = rng.standard_normal(6) * rng.uniform(0.1, 10)
        assert oracle.det3(g) == pytest.approx(np.linalg.det(_sym(g)), rel=1e-12, abs=1e-12)


def test_hessian_exact_on_quadratic():
    # centred differences are exact for quadratics: the discrete Hessian is A
    from paper_1411_7018_amd import problems as P
    p = P.quadratic(12, seed=7)
    for (i, j, k) in [(1, 1, 1), (5, 7, 3), (11, 11, 11), (6, 1, 10)]:
        g = oracle.hessian(p.u_exact, i, j, k)
        A = p.A
        want = [A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]]
        np.testing.assert_allclose(g, want, rtol=0, atol=1e-11)


def test_root_random_symmetric_vs_eigen_roots():
    """P6: smallest real root equals the minimum real root of
    prod(lambda_i - sigma) = F built from numpy eigenvalues; G - sigma* I is
    SPD; sigma* sits in the Theorem 2.2 bracket [l1 - F^{1/3}, l1)."""
    rng = np.random.default_rng(2)
    for trial in range(2000):
        scale = 10.0 ** rng.uniform(-2, 3)
        g = rng.standard_normal(6) * scale
        if trial % 3 == 0:                       # near-isotropic cases
            g[:3] = scale + 1e-3 * scale * rng.standard_normal(3)
            g[3:] *= 1e-3
        F = 10.0 ** rng.uniform(-3, 3) * scale ** 3
        lam = np.linalg.eigvalsh(_sym(g))
        e1, e2, e3 = lam.sum(), lam[0] * lam[1] + lam[0] * lam[2] + lam[1] * lam[2], lam.prod()
        # the smallest root is simple and below l1: bisection on (l1 - F^(1/3), l1)
        lo, hi = lam[0] - float(np.cbrt(F)) - 1e-12 * scale, lam[0]
        f = lambda s: np.prod(lam - s) - F   # noqa: E731
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if f(mid) > 0:
                lo = mid
            else:
                hi = mid
        want = 0.5 * (lo + hi)
        sig = oracle.local_root(g, F)
        tol = 1e-11 * (abs(lam).max() + float(np.cbrt(F)))
        assert abs(sig - want) <= tol, (trial, sig, want)
        # Theorem 2.2 bracket and convexity of the selected root
        assert lam[0] - float(np.cbrt(F)) - tol <= sig < lam[0] + tol
        assert np.all(lam - sig > -tol)
        # companion-matrix roots agree on the minimum real root
        cr = _min_real_root([-1.0, e1, -e2, e3 - F])
        assert abs(cr - want) <= 1e-6 * (abs(lam).max() + float(np.cbrt(F)))


def test_root_other_real_roots_not_convex():
    """Theorem 2.1: when three real roots exist only the smallest keeps the
    shifted Hessian positive definite."""
    rng = np.random.default_rng(3)
    seen = 0
    for _ in range(3000):
        lam = np.sort(rng.uniform(0.5, 5.0, 3))
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        G = Q @ np.diag(lam) @ Q.T
        g = [G[0, 0], G[1, 1], G[2, 2], G[0, 1], G[0, 2], G[1, 2]]
        F = rng.uniform(0.001, 0.3)
        roots = np.roots(np.poly(lam) * -1 + np.array([0, 0, 0, -F]))
        real = np.sort(roots[np.abs(roots.imag) < 1e-9].real)
        sig = oracle.local_root(g, F)
        assert sig == pytest.approx(real[0], abs=1e-9)
        if len(real) == 3:
            seen += 1
            for other in real[1:]:
                assert np.min(lam - other) < 0
    assert seen > 100


def test_root_isotropic_closed_form():
    """P7: G = mu I gives sigma* = mu - F^{1/3} (the p = 0 branch)."""
    for mu in (0.3, 1.0, 7.5, 123.0, -2.0):
        for F in (1e-6, 0.5, 1.0, 27.0, 1e4):
            g = [mu, mu, mu, 0.0, 0.0, 0.0]
            assert oracle.local_root(g, F) == pytest.approx(mu - float(np.cbrt(F)), rel=1e-14,
                                                            abs=1e-14 * (abs(mu) + 1))


def test_root_diagonal_product_of_factors():
    """P8: diagonal G (separable u): smallest root of prod(g_i - s) = F."""
    rng = np.random.default_rng(4)
    for _ in range(500):
        d = rng.uniform(-3, 10, 3)
        F = rng.uniform(0.01, 50)
        lo, hi = d.min() - float(np.cbrt(F)) - 1.0, d.min()
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if np.prod(d - mid) - F > 0:
                lo = mid
            else:
                hi = mid
        sig = oracle.local_root([d[0], d[1], d[2], 0, 0, 0], F)
        assert sig == pytest.approx(0.5 * (lo + hi), abs=1e-12 * (abs(d).max() + 1))


def test_root_nonpositive_F_takes_smallest_real_root():
    """Equation 2.9 applied literally when F <= 0 (coarse right-hand sides can
    dip): the minimum real root of the cubic."""
    rng = np.random.default_rng(5)
    for _ in range(500):
        g = rng.standard_normal(6) * 3
        F = -rng.uniform(0, 5) if rng.random() < 0.8 else 0.0
        lam = np.linalg.eigvalsh(_sym(g))
        want = _min_real_root(np.poly(lam) * -1 + np.array([0, 0, 0, -F]))
        sig = oracle.local_root(g, F)
        # check via the residual of the cubic and that no smaller real root exists
        assert abs(np.prod(lam - sig) - F) <= 1e-9 * (1 + abs(lam).max() ** 3)
        assert sig <= want + 1e-6 * (1 + abs(lam).max())


def test_single_unknown_grid_matches_expanded_cubic():
    """P5: on the 3^3 grid (h = 1/2, one unknown) one sweep returns the
    smallest real root of the paper's expanded P3 (eq. 2.8) in a, b, c, r, s, t."""
    rng = np.random.default_rng(6)
    h = 0.5
    for _ in range(300):
        u = rng.uniform(0.5, 2.0, (3, 3, 3))
        u += 0.5 * rng.uniform(0, 1) * np.fromfunction(
            lambda k, j, i: (i - 1.0) ** 2 + (j - 1.0) ** 2 + (k - 1.0) ** 2, (3, 3, 3))
        f = np.full((3, 3, 3), rng.uniform(0.05, 5.0))
        U = lambda i, j, k: u[1 + k, 1 + j, 1 + i]   # noqa: E731  offsets from centre
        a = U(1, 0, 0) + U(-1, 0, 0)
        b = U(0, 1, 0) + U(0, -1, 0)
        c = U(0, 0, 1) + U(0, 0, -1)
        r = 0.25 * (U(1, 1, 0) + U(-1, -1, 0) - U(-1, 1, 0) - U(1, -1, 0))
        s = 0.25 * (U(1, 0, 1) + U(-1, 0, -1) - U(-1, 0, 1) - U(1, 0, -1))
        t = 0.25 * (U(0, 1, 1) + U(0, -1, -1) - U(0, 1, -1) - U(0, -1, 1))
        coeffs = [-8.0, 4.0 * (a + b + c), 2.0 * (r * r + s * s + t * t - a * b - a * c - b * c),
                  a * b * c - a * t * t - b * s * s - c * r * r + 2 * r * s * t - h ** 6 * f[1, 1, 1]]
        want = _min_real_root(coeffs)
        v = u.copy()
        oracle.sweep(v, f, "4c")
        assert v[1, 1, 1] == pytest.approx(want, rel=1e-10, abs=1e-12)
        mask = np.ones_like(u, bool)
        mask[1, 1, 1] = False
        assert np.array_equal(v[mask], u[mask])   # Dirichlet layer untouched


def _bisect_double(l1, l3, F):
    """Smallest root of (l1 - s)^2 (l3 - s) = F below l1 by bisection on the
    product form (no cancellation)."""
    lo, hi = l1 - 1.0 - abs(F) ** (1.0 / 3.0), l1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (l1 - mid) ** 2 * (l3 - mid) - F > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("F", [1e-300, 1e-20, 1e-12, 1e-6])
def test_root_double_smallest_eigenvalue_tiny_F(F):
    """G = diag(1, 1, 2): a double smallest eigenvalue.  For F > 0 the cubic
    has three real roots, the lower two within ~sqrt(F) of 1 (Theorem 2.2:
    the wanted one lies below lambda_min).  Rounding hides the separation
    of the lower pair from the discriminant, which must not turn the result
    into the largest root (near 2).  Near a double root the cubic in its
    expanded or shifted form is flat to second order, so rounding errors of
    size eps in q move the root by ~sqrt(eps): the tolerance is 3e-8."""
    g = np.array([1.0, 1.0, 2.0, 0.0, 0.0, 0.0])
    want = _bisect_double(1.0, 2.0, F)
    got = oracle.local_root(g, F)
    assert got <= 1.0 + 1e-12
    assert got == pytest.approx(want, abs=3e-8)
