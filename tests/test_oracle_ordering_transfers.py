"""Pins for the orderings (Section 2: four or more colours decouple the
19-point stencil) and the transfer operators of Section 3."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P

STENCIL = [d for d in itertools.product((-1, 0, 1), repeat=3)
           if d != (0, 0, 0) and sum(abs(x) for x in d) <= 2]   # 6 faces + 12 edges


def test_stencil_has_19_points():
    assert len(STENCIL) + 1 == 19


@pytest.mark.parametrize("order,ncol", [("4c", 4), ("8c", 8)])
def test_coloring_decouples_19_point_stencil(order, ncol):
    """P9: no two stencil neighbours share a colour (brute force on 6^3)."""
    n = 6
    conflicts = 0
    seen = set()
    for k, j, i in itertools.product(range(n), repeat=3):
        c = oracle.color(order, i, j, k)
        seen.add(c)
        for dx, dy, dz in STENCIL:
            conflicts += oracle.color(order, i + dx, j + dy, k + dz) == c
    assert conflicts == 0
    assert seen == set(range(ncol))


def test_red_black_does_not_decouple():
    """Two colours leave every edge neighbour in the same colour: 12 per node."""
    per_node = sum(1 for d in STENCIL if sum(d) % 2 == 0)
    assert per_node == 12


def test_no_linear_mod4_coloring_decouples():
    for a, b, c in itertools.product(range(4), repeat=3):
        if all((a * dx + b * dy + c * dz) % 4 != 0 for dx, dy, dz in STENCIL):
            pytest.fail(f"linear colouring {(a, b, c)} unexpectedly works")


@pytest.mark.parametrize("order", ["4c", "8c"])
def test_colour_phase_independent_of_same_colour_nodes(order):
    """Bitwise: perturbing other nodes of the colour being updated does not
    change any update of that phase, so in-place updates within a colour are
    race-free in any order."""
    n = 10
    p = P.exp_cos(n, seed=11)
    rng = np.random.default_rng(0)
    base = p.u_exact + 0.01 * rng.standard_normal(p.u_exact.shape)
    base = P.initial_guess(p, base)
    K, J, I = np.meshgrid(*(np.arange(n + 1),) * 3, indexing="ij")
    col = np.vectorize(lambda i, j, k: oracle.color(order, i, j, k))(I, J, K)
    inner = np.zeros_like(base, bool)
    inner[1:-1, 1:-1, 1:-1] = True
    for c in range(4 if order == "4c" else 8):
        clean = base.copy()
        oracle.sweep_color(clean, p.f, c, order)
        sel = (col == c) & inner
        perturb = sel & (rng.random(base.shape) < 0.5)
        pert = base.copy()
        pert[perturb] += 0.05
        oracle.sweep_color(pert, p.f, c, order)
        keep = sel & ~perturb
        assert np.array_equal(clean[keep], pert[keep])
        assert np.array_equal(clean[~sel], base[~sel])


def _coarse_coords(nc):
    t = np.arange(nc + 1) / nc
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    return X, Y, Z


@pytest.mark.parametrize("rmode", [oracle.RESTRICT_HALF, oracle.RESTRICT_FULL])
def test_restriction_preserves_constants_and_linears(rmode):
    """P10: both residual restrictions have weights summing to one and are
    symmetric, so constants and linear functions restrict exactly."""
    nf = 12
    x, y, z = P.grid(nf)
    rf = 0.3 + 1.5 * x - 0.7 * y + 2.0 * z
    uf = np.zeros_like(rf)            # S_H(0) = 0 for the Laplacian
    wc, bc = oracle.restrict(uf, rf, op="lap", rmode=rmode)
    X, Y, Z = _coarse_coords(nf // 2)
    want = 0.3 + 1.5 * X - 0.7 * Y + 2.0 * Z
    np.testing.assert_allclose(bc[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1], rtol=0, atol=1e-14)
    assert np.all(bc[0] == 0) and np.all(bc[:, :, -1] == 0)


def test_full_weighting_kills_single_direction_oscillation():
    """The 27-point full weighting annihilates (-1)^i (any single-axis
    highest-frequency mode); half-weighting passes 2/3 of it."""
    nf = 12
    K, J, I = np.meshgrid(*(np.arange(nf + 1),) * 3, indexing="ij")
    rf = (-1.0) ** I
    uf = np.zeros_like(rf)
    _, b_full = oracle.restrict(uf, rf, op="lap", rmode=oracle.RESTRICT_FULL)
    _, b_half = oracle.restrict(uf, rf, op="lap", rmode=oracle.RESTRICT_HALF)
    assert np.abs(b_full[1:-1, 1:-1, 1:-1]).max() == 0.0
    np.testing.assert_allclose(b_half[1:-1, 1:-1, 1:-1], 8.0 / 12.0, rtol=1e-15)


def test_injection_and_coarse_operator():
    """w_H is the injection (boundary included) and b_H = S_H(w_H) + r_H with
    S_H the same discretisation at step 2h (exact on quadratics)."""
    p = P.quadratic(16, seed=3)
    rf = np.zeros_like(p.u_exact)
    wc, bc = oracle.restrict(p.u_exact, rf, op="ma")
    np.testing.assert_array_equal(wc, p.u_exact[::2, ::2, ::2])
    np.testing.assert_allclose(bc[1:-1, 1:-1, 1:-1], np.linalg.det(p.A), rtol=1e-12)


def test_trilinear_prolongation_reproduces_trilinear_functions():
    """P10: u_h += I_H^h (u_H - w_H) is exact for trilinear corrections
    (weights 1, 1/2, 1/4, 1/8: the 1/64 prefactor read as 1/8)."""
    nf = 12
    nc = nf // 2
    X, Y, Z = _coarse_coords(nc)
    e = lambda x, y, z: (1 + 2 * x) * (2 - y) * (0.5 + z) + 3 * x * y - z   # noqa: E731
    uc = e(X, Y, Z)
    wc = np.zeros_like(uc)
    uc[0], uc[-1] = 0, 0                   # the correction vanishes on the boundary
    uc[:, 0], uc[:, -1], uc[:, :, 0], uc[:, :, -1] = 0, 0, 0, 0
    uf = np.zeros((nf + 1,) * 3)
    oracle.prolong_correct(uf, uc, wc)
    x, y, z = P.grid(nf)
    want = e(x, y, z)
    inner = (slice(2, -2),) * 3           # nodes whose coarse cell has no boundary corner
    np.testing.assert_allclose(uf[inner], want[inner], rtol=0, atol=1e-13)
    assert np.all(uf[0] == 0) and np.all(uf[:, -1] == 0)


def test_prolongation_constant_and_weights_sum():
    nf = 8
    uc = np.zeros((nf // 2 + 1,) * 3)
    uc[1:-1, 1:-1, 1:-1] = 1.0
    wc = np.zeros_like(uc)
    uf = np.zeros((nf + 1,) * 3)
    oracle.prolong_correct(uf, uc, wc)
    # fine node (3,3,3) lies in a cell whose 8 corners are coarse interior nodes
    assert uf[3, 3, 3] == 1.0
    # fine node (1,1,1): one of 8 corners is interior -> weight 1/8
    assert uf[1, 1, 1] == 0.125
    assert uf[2, 2, 1] == 0.5 and uf[2, 1, 1] == 0.25
