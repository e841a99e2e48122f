"""CPU oracle for the 3D Monge-Ampere FAS multigrid method (serial, FP64).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product library never
imports, links or calls it, and it shares no code with the HIP path.

The arithmetic lives in ``ma_oracle.c`` (plain C, ``-O2 -ffp-contract=off``);
this module compiles it on demand and marshals numpy arrays through ctypes.
Every array is an (n+1, n+1, n+1) C-contiguous float64 array indexed
[k, j, i] (x fastest), as in Section 2 of the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ma_oracle.c")
_SRC2 = os.path.join(_HERE, "ma2_oracle.c")    # the 2D variant (oracle.ma2)
_LIB = os.path.join(_HERE, "libmaoracle.so")

ORDER_4C, ORDER_8C, ORDER_LEX = 0, 1, 2
_ORDERS = {"4c": 0, "color4": 0, "8c": 1, "color8": 1, "lex": 2}


def build(force: bool = True) -> str:
    """Compile ma_oracle.c and ma2_oracle.c into libmaoracle.so next to them."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
               "-D_GNU_SOURCE", "-Wall", "-o", _LIB + ".tmp", _SRC, _SRC2, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("nu0", ctypes.c_int),
                ("order", ctypes.c_int), ("rmode", ctypes.c_int),
                ("max_cycles", ctypes.c_int),
                ("tol", ctypes.c_double), ("init", ctypes.c_int),
                ("init_tol", ctypes.c_double), ("init_max_cycles", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("init_cycles", ctypes.c_int),
                ("converged", ctypes.c_int), ("res0", ctypes.c_double),
                ("res", ctypes.c_double), ("seconds", ctypes.c_double),
                ("nonconvex", ctypes.c_long)]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.mao_levels.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.mao_hessian.argtypes = [ctypes.c_int, _DP, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, _DP]
        L.mao_det3.argtypes = [_DP]
        L.mao_det3.restype = ctypes.c_double
        L.mao_local_root.argtypes = [_DP, ctypes.c_double]
        L.mao_local_root.restype = ctypes.c_double
        L.mao_color.argtypes = [ctypes.c_int] * 4
        L.mao_sweep.argtypes = [ctypes.c_int, _DP, _DP, ctypes.c_int]
        L.mao_sweep.restype = ctypes.c_long
        L.mao_sweep_color.argtypes = [ctypes.c_int, _DP, _DP, ctypes.c_int, ctypes.c_int]
        L.mao_sweep_color.restype = ctypes.c_long
        L.mao_poisson_sweep.argtypes = [ctypes.c_int, _DP, _DP, ctypes.c_int]
        L.mao_residual.argtypes = [ctypes.c_int, _DP, _DP, _DP]
        L.mao_residual.restype = ctypes.c_double
        L.mao_poisson_residual.argtypes = [ctypes.c_int, _DP, _DP, _DP]
        L.mao_poisson_residual.restype = ctypes.c_double
        L.mao_restrict.argtypes = [ctypes.c_int, _DP, _DP, _DP, _DP, ctypes.c_int,
                                   ctypes.c_int]
        L.mao_prolong_correct.argtypes = [ctypes.c_int, _DP, _DP, _DP]
        L.mao_poisson_rhs.argtypes = [ctypes.c_int, _DP, _DP]
        L.mao_vcycle.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(Params)]
        L.mao_vcycle.restype = ctypes.c_long
        L.mao_poisson_vcycle.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(Params)]
        L.mao_poisson_init.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(Params)]
        L.mao_solve.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(Params),
                                ctypes.POINTER(Report), _DP, ctypes.c_int]
        L.mao_inject.argtypes = [ctypes.c_int, _DP, _DP]
        L.mao_inject.restype = None
        L.mao_fmg_interp.argtypes = [ctypes.c_int, _DP, _DP]
        L.mao_fmg_interp.restype = None
        L.mao_fmg.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(Params)]
        L.mao_fmg.restype = ctypes.c_long
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
        raise TypeError("oracle arrays must be C-contiguous float64")
    return a.ctypes.data_as(_DP)


def _n_of(a: np.ndarray) -> int:
    if a.ndim != 3 or not (a.shape[0] == a.shape[1] == a.shape[2]):
        raise ValueError("grid arrays are (n+1, n+1, n+1)")
    return a.shape[0] - 1


def _order(order) -> int:
    return _ORDERS[order] if isinstance(order, str) else int(order)


RESTRICT_HALF, RESTRICT_FULL = 0, 1


def default_rmode(order) -> int:
    """Half-weighting for the lexicographic ordering (the paper's pairing),
    full weighting for the multicolour orderings."""
    return RESTRICT_HALF if _order(order) == ORDER_LEX else RESTRICT_FULL


INIT_NONE, INIT_POISSON, INIT_FMG = 0, 1, 2


def params(nu1=2, nu2=2, nu0=1, order="4c", max_cycles=100, tol=1e-10, init=True,
           init_tol=1e-6, init_max_cycles=30, rmode=None) -> Params:
    """init: True / "poisson" (Poisson guess), "fmg" (one FMG-FAS iteration,
    Algorithm 2, counted as the first cycle) or False / "none"."""
    rm = default_rmode(order) if rmode is None else int(rmode)
    if init is True or init == "poisson":
        iv = INIT_POISSON
    elif init == "fmg":
        iv = INIT_FMG
    else:
        iv = INIT_NONE
    return Params(nu1, nu2, nu0, _order(order), rm, max_cycles, tol, iv,
                  init_tol, init_max_cycles)


def levels(n: int):
    buf = (ctypes.c_int * 32)()
    L = lib().mao_levels(n, buf, 32)
    return [buf[i] for i in range(L)]


def hessian(u: np.ndarray, i: int, j: int, k: int) -> np.ndarray:
    g = np.zeros(6)
    lib().mao_hessian(_n_of(u), _ptr(u), i, j, k, _ptr(g))
    return g


def det3(g) -> float:
    g = np.ascontiguousarray(g, dtype=np.float64)
    return lib().mao_det3(_ptr(g))


def local_root(g, F: float) -> float:
    """Smallest real root sigma of det(G - sigma I) = F, G = (xx,yy,zz,xy,xz,yz)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    return lib().mao_local_root(_ptr(g), float(F))


def color(order, i, j, k) -> int:
    return lib().mao_color(_order(order), i, j, k)


def sweep(u: np.ndarray, F: np.ndarray, order="4c") -> int:
    """One nonlinear GS sweep in place; returns # non-certified updates."""
    return lib().mao_sweep(_n_of(u), _ptr(u), _ptr(F), _order(order))


def sweep_color(u: np.ndarray, F: np.ndarray, c: int, order="4c") -> int:
    return lib().mao_sweep_color(_n_of(u), _ptr(u), _ptr(F), _order(order), c)


def poisson_sweep(u: np.ndarray, R: np.ndarray, order="4c") -> None:
    lib().mao_poisson_sweep(_n_of(u), _ptr(u), _ptr(R), _order(order))


def residual(u: np.ndarray, F: np.ndarray, out: bool = True):
    """(r, sum r^2) with r = F - det(D^2_h u) inside and 0 on the boundary."""
    r = np.zeros_like(u) if out else None
    ss = lib().mao_residual(_n_of(u), _ptr(u), _ptr(F), _ptr(r) if out else None)
    return r, ss


def poisson_residual(u: np.ndarray, R: np.ndarray):
    r = np.zeros_like(u)
    ss = lib().mao_poisson_residual(_n_of(u), _ptr(u), _ptr(R), _ptr(r))
    return r, ss


def l2(ss: float, n: int) -> float:
    """Discrete L2 norm sqrt(h^3 sum r^2)."""
    return float(np.sqrt(ss / float(n) ** 3))


def restrict(uf: np.ndarray, rf: np.ndarray, op: str = "ma", rmode: int = RESTRICT_FULL):
    """FAS restriction: (w_H = injection of uf, b_H = S_H(w_H) + I_h^H rf)."""
    nf = _n_of(uf)
    if nf % 2:
        raise ValueError("fine n must be even")
    nc = nf // 2
    wc = np.zeros((nc + 1,) * 3)
    bc = np.zeros((nc + 1,) * 3)
    lib().mao_restrict(nf, _ptr(uf), _ptr(rf), _ptr(wc), _ptr(bc), 0 if op == "ma" else 1,
                       int(rmode))
    return wc, bc


def prolong_correct(uf: np.ndarray, uc: np.ndarray, wc: np.ndarray) -> None:
    lib().mao_prolong_correct(_n_of(uf), _ptr(uf), _ptr(uc), _ptr(wc))


def inject(vf: np.ndarray) -> np.ndarray:
    """Injection onto the grid with half the intervals (every coarse node)."""
    nf = _n_of(vf)
    vc = np.empty((nf // 2 + 1,) * 3)
    lib().mao_inject(nf, _ptr(vf), _ptr(vc))
    return vc


def fmg_interp(uc: np.ndarray, uf: np.ndarray) -> None:
    """FMG interpolation of the coarse uc into the interior of uf."""
    nc = _n_of(uc)
    if _n_of(uf) != 2 * nc:
        raise ValueError("uf must have twice the intervals of uc")
    lib().mao_fmg_interp(nc, _ptr(uc), _ptr(uf))


def fmg(u: np.ndarray, f: np.ndarray, p: Params | None = None) -> int:
    """One FMG-FAS iteration (Algorithm 2) in place; u's interior is ignored."""
    p = p or params()
    nc = lib().mao_fmg(_n_of(u), _ptr(u), _ptr(f), ctypes.byref(p))
    if nc < 0:
        raise MemoryError("oracle allocation failed")
    return nc


def poisson_rhs(f: np.ndarray) -> np.ndarray:
    R = np.empty_like(f)
    lib().mao_poisson_rhs(_n_of(f), _ptr(f), _ptr(R))
    return R


def vcycle(u: np.ndarray, f: np.ndarray, p: Params | None = None) -> int:
    p = p or params()
    nc = lib().mao_vcycle(_n_of(u), _ptr(u), _ptr(f), ctypes.byref(p))
    if nc < 0:
        raise MemoryError("oracle allocation failed")
    return nc


def poisson_vcycle(u: np.ndarray, R: np.ndarray, p: Params | None = None) -> None:
    p = p or params()
    if lib().mao_poisson_vcycle(_n_of(u), _ptr(u), _ptr(R), ctypes.byref(p)) < 0:
        raise MemoryError("oracle allocation failed")


def poisson_init(u: np.ndarray, f: np.ndarray, p: Params | None = None) -> int:
    p = p or params()
    c = lib().mao_poisson_init(_n_of(u), _ptr(u), _ptr(f), ctypes.byref(p))
    if c < 0:
        raise MemoryError("oracle allocation failed")
    return c


def solve(u: np.ndarray, f: np.ndarray, p: Params | None = None, hist_cap: int = 200):
    """Solve in place; returns (status, Report, residual history)."""
    p = p or params()
    rep = Report()
    hist = np.zeros(hist_cap)
    st = lib().mao_solve(_n_of(u), _ptr(u), _ptr(f), ctypes.byref(p), ctypes.byref(rep),
                         _ptr(hist), hist_cap)
    if st < 0:
        raise MemoryError("oracle allocation failed")
    return st, rep, hist[: min(rep.cycles, hist_cap)].copy()


def solve_limit(u: np.ndarray, f: np.ndarray, max_cycles: int = 200, **kw):
    """Run V-cycles until the residual stagnates on its round-off floor."""
    p = params(tol=-1.0, max_cycles=max_cycles, **kw)
    return solve(u, f, p)
