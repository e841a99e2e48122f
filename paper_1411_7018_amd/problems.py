"""Seeded synthetic inputs for the 3D Monge-Ampere Dirichlet problem.

This module only builds problem data: grid coordinates, an analytic solution
``u`` (whose values on the boundary layer are the Dirichlet data g) and the
matching right-hand side ``f = det(Hess u)`` evaluated from the analytic
Hessian.  It contains none of the discrete method (no stencil, no root
selection, no transfer); both the CPU oracle and the HIP path consume the
arrays it returns.

Grid convention (Section 2, discretisation of the unit cube): h = 1/N, nodes
x_i = i h for i = 0..N, Dirichlet nodes are those with any index in {0, N};
arrays have shape (N+1, N+1, N+1) indexed [k, j, i] so that the C-order
flattening puts x fastest.

Workloads:
  * ``example4``      -- Example 4 of Section 4 (u = exp(|x|^2/2)).
  * ``example5`` .. ``example7`` -- Examples 5-7 of Section 4 (Example 5's
                         (0, pi)^3 restated on the unit cube).
  * ``quadratic``     -- u = x^T A x / 2 + b^T x with a seeded SPD A whose
                         eigenvalues lie in [0.5, 2] and b ~ U[-1, 1]^3;
                         centred differences are exact on quadratics.
  * ``exp_cos``       -- exp(|x|^2/2) plus six seeded low-frequency cosines
                         scaled so that Hess u >= 0.5 I everywhere.
  * ``figure1_error`` -- the oscillating error field of Figure 1.
  * ``batch_specs`` / ``arrival_trace`` -- the mixed-size batch and the
                         Poisson-arrival request stream.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "grid", "example4", "example5", "example6", "example7", "quadratic", "exp_cos",
    "make", "make_device",
    "figure1_error", "initial_guess", "batch_specs", "arrival_trace",
    "SERVE_SIZES", "SERVE_WEIGHTS", "BATCH_SIZES",
]

BATCH_SIZES = (32, 64, 96, 128)          # 33^3, 65^3, 97^3, 129^3 grids
SERVE_SIZES = (64, 128, 256, 384)        # 65^3 ... 385^3 grids
SERVE_WEIGHTS = (0.4, 0.3, 0.2, 0.1)


@dataclasses.dataclass
class Problem:
    """One Dirichlet problem on the (N+1)^3 unit-cube grid."""
    name: str
    n: int
    f: np.ndarray          # (N+1)^3 float64, right-hand side at every node
    u_exact: np.ndarray    # (N+1)^3 float64, analytic solution (boundary = g)

    @property
    def h(self) -> float:
        return 1.0 / self.n


def grid(n: int):
    """Coordinates x, y, z of the (n+1)^3 nodes, each shaped [k, j, i]."""
    if n < 2:
        raise ValueError("n must be >= 2")
    t = np.arange(n + 1, dtype=np.float64) / n
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return x, y, z


def example4(n: int) -> Problem:
    """Example 4: u = exp(|x|^2/2), f = (1 + |x|^2) exp(3|x|^2/2)."""
    x, y, z = grid(n)
    r2 = x * x + y * y + z * z
    u = np.exp(0.5 * r2)
    f = (1.0 + r2) * np.exp(1.5 * r2)
    return Problem("example4", n, f, u)


def _random_spd(rng: np.random.Generator) -> np.ndarray:
    """A = Q diag(lam) Q^T, Q from a sign-fixed QR of a 3x3 normal sample."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    lam = rng.uniform(0.5, 2.0, size=3)
    return (q * lam[None, :]) @ q.T


def _quadratic_params(seed: int):
    rng = np.random.default_rng(seed)
    a = _random_spd(rng)
    a = 0.5 * (a + a.T)
    b = rng.uniform(-1.0, 1.0, size=3)
    return a, b


def quadratic(n: int, seed: int = 0) -> Problem:
    """u = x^T A x / 2 + b^T x with seeded SPD A (eigenvalues in [0.5, 2])."""
    a, b = _quadratic_params(seed)
    x, y, z = grid(n)
    u = (0.5 * (a[0, 0] * x * x + a[1, 1] * y * y + a[2, 2] * z * z)
         + a[0, 1] * x * y + a[0, 2] * x * z + a[1, 2] * y * z
         + b[0] * x + b[1] * y + b[2] * z)
    f = np.full_like(u, float(np.linalg.det(a)))
    p = Problem("quadratic", n, f, u)
    p.A, p.b = a, b          # kept for tests
    return p


def _cos_terms(rng: np.random.Generator, count: int = 6):
    """Wave vectors k in {0,1,2}^3 \\ {0}, phases and amplitudes."""
    ks = []
    while len(ks) < count:
        k = rng.integers(0, 3, size=3)
        if k.any():
            ks.append(k.astype(np.float64))
    ks = np.array(ks)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=count)
    c = rng.uniform(-1.0, 1.0, size=count)
    # 0.1 * sum |c_m| pi^2 |k_m|^2 <= 0.5 bounds the spectral norm of the
    # cosine part of the Hessian by 0.5, while Hess exp(|x|^2/2) >= I.
    budget = 0.1 * np.sum(np.abs(c) * math.pi ** 2 * np.sum(ks * ks, axis=1))
    if budget > 0.5:
        c = c * (0.5 / budget)
    return ks, phi, c


def exp_cos(n: int, seed: int = 0) -> Problem:
    """u = exp(|x|^2/2) + 0.1 sum_m c_m cos(pi k_m.x + phi_m); f analytic."""
    rng = np.random.default_rng(seed)
    ks, phi, c = _cos_terms(rng)
    x, y, z = grid(n)
    X = (x, y, z)
    r2 = x * x + y * y + z * z
    e = np.exp(0.5 * r2)
    u = e.copy()
    # Hessian of exp(|x|^2/2) is e (I + x x^T).
    H = [[e * ((1.0 if a == b else 0.0) + X[a] * X[b]) for b in range(3)]
         for a in range(3)]
    for m in range(len(c)):
        arg = math.pi * (ks[m, 0] * x + ks[m, 1] * y + ks[m, 2] * z) + phi[m]
        cm = 0.1 * c[m]
        u += cm * np.cos(arg)
        w = -cm * math.pi ** 2 * np.cos(arg)
        for a in range(3):
            for b in range(3):
                H[a][b] = H[a][b] + w * ks[m, a] * ks[m, b]
    f = (H[0][0] * H[1][1] * H[2][2] + 2.0 * H[0][1] * H[1][2] * H[0][2]
         - H[0][0] * H[1][2] ** 2 - H[1][1] * H[0][2] ** 2
         - H[2][2] * H[0][1] ** 2)
    return Problem("exp_cos", n, f, u)


def example5(n: int) -> Problem:
    """Example 5 on (0, pi)^3: u = -sum sin(x_i) + |x|^2/2, whose Hessian is
    diag(1 + sin x_i), f = prod(1 + sin x_i).  Stated on the unit cube by
    x = pi xi: the grid values of u are those of u(pi xi), and since every
    discrete second difference on the (0, pi)^3 grid is pi^-2 times the one
    on the unit-cube grid, the discrete equations are those of the unit
    cube with f scaled by pi^6 (the Newton roots scale by pi^2 and the
    updates u_p + sigma h^2 / 2 coincide)."""
    x, y, z = grid(n)
    X, Y, Z = math.pi * x, math.pi * y, math.pi * z
    u = -np.sin(X) - np.sin(Y) - np.sin(Z) + 0.5 * (X * X + Y * Y + Z * Z)
    f = math.pi ** 6 * (np.sin(X) + 1.0) * (np.sin(Y) + 1.0) * (np.sin(Z) + 1.0)
    return Problem("example5", n, f, u)


def example6(n: int) -> Problem:
    """Example 6: u = |x|^{3/2} / 3, f = |x|^{-3/2} / 16, singular at the
    origin (a boundary node, where f is never read and is set to 0)."""
    x, y, z = grid(n)
    r2 = x * x + y * y + z * z
    u = r2 ** 0.75 / 3.0
    with np.errstate(divide="ignore"):
        f = np.where(r2 > 0.0, r2 ** -0.75 / 16.0, 0.0)
    return Problem("example6", n, f, u)


def example7(n: int) -> Problem:
    """Example 7: u = -sqrt(3 - |x|^2), f = 3 (3 - |x|^2)^{-5/2}; the
    gradient is unbounded at the corner (1, 1, 1) (a boundary node, where f
    is never read and is set to 0)."""
    x, y, z = grid(n)
    q = 3.0 - (x * x + y * y + z * z)
    q = np.maximum(q, 0.0)
    u = -np.sqrt(q)
    with np.errstate(divide="ignore"):
        f = np.where(q > 0.0, 3.0 * q ** -2.5, 0.0)
    return Problem("example7", n, f, u)


def make(kind: str, n: int, seed: int = 0) -> Problem:
    if kind == "example4":
        return example4(n)
    if kind == "example5":
        return example5(n)
    if kind == "example6":
        return example6(n)
    if kind == "example7":
        return example7(n)
    if kind == "quadratic":
        return quadratic(n, seed)
    if kind == "exp_cos":
        return exp_cos(n, seed)
    raise ValueError(f"unknown problem kind {kind!r}")


def figure1_error(n: int) -> np.ndarray:
    """Figure 1 initial error sin(pi x)sin(pi y)sin(pi z) + 0.5 sin(15 pi .)^3."""
    x, y, z = grid(n)
    p = math.pi
    return (np.sin(p * x) * np.sin(p * y) * np.sin(p * z)
            + 0.5 * np.sin(15 * p * x) * np.sin(15 * p * y) * np.sin(15 * p * z))


def initial_guess(p: Problem, interior: float | np.ndarray = 0.0) -> np.ndarray:
    """Array holding g on the Dirichlet layer and ``interior`` inside."""
    u = np.empty_like(p.u_exact)
    u[...] = interior
    u[0, :, :] = p.u_exact[0, :, :]
    u[-1, :, :] = p.u_exact[-1, :, :]
    u[:, 0, :] = p.u_exact[:, 0, :]
    u[:, -1, :] = p.u_exact[:, -1, :]
    u[:, :, 0] = p.u_exact[:, :, 0]
    u[:, :, -1] = p.u_exact[:, :, -1]
    return u


def batch_specs(count: int = 64, seed: int = 4000):
    """Seeded (kind, n, seed) triples: sizes uniform over BATCH_SIZES,
    quadratic or exp-cos data with probability 1/2 each."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(seed + s)
        n = int(rng.choice(BATCH_SIZES))
        kind = "quadratic" if rng.random() < 0.5 else "exp_cos"
        out.append((kind, n, seed + s))
    return out


def arrival_trace(count: int, rate: float, seed: int = 5000):
    """Poisson arrivals: (t_arrival_seconds, kind, n, seed) for each request,
    sizes drawn from SERVE_SIZES with SERVE_WEIGHTS."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    sizes = rng.choice(SERVE_SIZES, size=count, p=SERVE_WEIGHTS)
    kinds = np.where(rng.random(count) < 0.5, "quadratic", "exp_cos")
    return [(float(t[i]), str(kinds[i]), int(sizes[i]), seed + 1 + i)
            for i in range(count)]


def make_device(kind: str, n: int, seed: int = 0, device="cuda", exact: bool = False):
    """The problem of ``make(kind, n, seed)`` evaluated with torch on
    ``device`` (float64): returns (u0, f) -- u0 holds g on the Dirichlet
    layer and 0 inside -- plus u_exact when ``exact``.  Same seeded
    parameters and formulas as the numpy generators; values can differ from
    them in the last bits (device exp / cos).  For large served requests,
    where building the data on the host would dominate."""
    import torch

    t = torch.arange(n + 1, dtype=torch.float64, device=device) / n
    z, y, x = torch.meshgrid(t, t, t, indexing="ij")
    r2 = x * x + y * y + z * z
    if kind == "example4":
        u = torch.exp(0.5 * r2)
        f = (1.0 + r2) * torch.exp(1.5 * r2)
    elif kind == "example5":
        X, Y, Z = math.pi * x, math.pi * y, math.pi * z
        u = -torch.sin(X) - torch.sin(Y) - torch.sin(Z) + 0.5 * (X * X + Y * Y + Z * Z)
        f = math.pi ** 6 * (torch.sin(X) + 1.0) * (torch.sin(Y) + 1.0) * (torch.sin(Z) + 1.0)
    elif kind == "example6":
        u = r2 ** 0.75 / 3.0
        f = torch.where(r2 > 0.0, r2.clamp_min(1e-300) ** -0.75 / 16.0, torch.zeros_like(r2))
    elif kind == "example7":
        q = (3.0 - r2).clamp_min(0.0)
        u = -torch.sqrt(q)
        f = torch.where(q > 0.0, 3.0 * q.clamp_min(1e-300) ** -2.5, torch.zeros_like(q))
    elif kind == "quadratic":
        a, b = _quadratic_params(seed)
        u = (0.5 * (a[0, 0] * x * x + a[1, 1] * y * y + a[2, 2] * z * z)
             + a[0, 1] * x * y + a[0, 2] * x * z + a[1, 2] * y * z
             + b[0] * x + b[1] * y + b[2] * z)
        f = torch.full_like(u, float(np.linalg.det(a)))
    elif kind == "exp_cos":
        ks, phi, c = _cos_terms(np.random.default_rng(seed))
        X = (x, y, z)
        e = torch.exp(0.5 * r2)
        u = e.clone()
        H = [[e * ((1.0 if p == q else 0.0) + X[p] * X[q]) for q in range(3)] for p in range(3)]
        for m in range(len(c)):
            arg = math.pi * (ks[m, 0] * x + ks[m, 1] * y + ks[m, 2] * z) + phi[m]
            ca = torch.cos(arg)
            cm = 0.1 * c[m]
            u += cm * ca
            w = (-cm * math.pi ** 2) * ca
            for p in range(3):
                for q in range(3):
                    if ks[m, p] * ks[m, q] != 0.0:
                        H[p][q] = H[p][q] + w * (ks[m, p] * ks[m, q])
        f = (H[0][0] * H[1][1] * H[2][2] + 2.0 * H[0][1] * H[1][2] * H[0][2]
             - H[0][0] * H[1][2] ** 2 - H[1][1] * H[0][2] ** 2
             - H[2][2] * H[0][1] ** 2)
        del H, e
    else:
        raise ValueError(f"unknown problem kind {kind!r}")
    del x, y, z, r2
    u0 = u.clone()
    u0[1:-1, 1:-1, 1:-1] = 0.0
    if exact:
        return u0, f, u
    return u0, f


# ---------------------------------------------------------------------------
# 2D variant (u_xx u_yy - u_xy^2 = f on the unit square), Examples 1-3 of
# Section 4.  Arrays (n+1, n+1) indexed [j, i], x fastest.
# ---------------------------------------------------------------------------
def grid2(n: int):
    if n < 2:
        raise ValueError("n must be >= 2")
    t = np.arange(n + 1, dtype=np.float64) / n
    y, x = np.meshgrid(t, t, indexing="ij")
    return x, y


def example2d(number: int, n: int) -> Problem:
    """Example 1: u = exp(|x|^2/2), f = (1 + |x|^2) exp(|x|^2);
    Example 2: u = (2 sqrt 2 / 3) |x|^{3/2}, f = 1/|x| (singular at the
    origin, a boundary node where f is never read and is set to 0);
    Example 3: u = -sqrt(2 - |x|^2), f = 2 / (2 - |x|^2)^2 (unbounded
    gradient at the corner (1, 1), where f is set to 0)."""
    x, y = grid2(n)
    r2 = x * x + y * y
    if number == 1:
        u = np.exp(0.5 * r2)
        f = (1.0 + r2) * np.exp(r2)
    elif number == 2:
        u = (2.0 * math.sqrt(2.0) / 3.0) * r2 ** 0.75
        with np.errstate(divide="ignore"):
            f = np.where(r2 > 0.0, 1.0 / np.sqrt(np.where(r2 > 0.0, r2, 1.0)), 0.0)
    elif number == 3:
        q = np.maximum(2.0 - r2, 0.0)
        u = -np.sqrt(q)
        with np.errstate(divide="ignore"):
            f = np.where(q > 0.0, 2.0 / np.where(q > 0.0, q, 1.0) ** 2, 0.0)
    else:
        raise ValueError("2D examples are 1, 2, 3")
    return Problem(f"example2d_{number}", n, f, u)


def initial_guess2(p: Problem, interior: float | np.ndarray = 0.0) -> np.ndarray:
    u = np.empty_like(p.u_exact)
    u[...] = interior
    u[0, :] = p.u_exact[0, :]
    u[-1, :] = p.u_exact[-1, :]
    u[:, 0] = p.u_exact[:, 0]
    u[:, -1] = p.u_exact[:, -1]
    return u
