"""CPU oracle for the 2D variant (u_xx u_yy - u_xy^2 = f), serial FP64.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the arithmetic is in
``ma2_oracle.c``; arrays are (n+1, n+1) C-contiguous float64 indexed [j, i]
(x fastest).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import lib as _lib3

_DP = ctypes.POINTER(ctypes.c_double)
ORDERS = {"4c": 0, "rb": 1, "lex": 2}
_ready = False


class Params(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("nu0", ctypes.c_int),
                ("order", ctypes.c_int), ("rmode", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("tol", ctypes.c_double), ("init", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("converged", ctypes.c_int),
                ("res0", ctypes.c_double), ("res", ctypes.c_double),
                ("nonconvex", ctypes.c_long)]


def lib():
    global _ready
    L = _lib3()
    if not _ready:
        L.ma2_levels.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.ma2_hessian.argtypes = [ctypes.c_int, _DP, ctypes.c_int, ctypes.c_int, _DP]
        L.ma2_hessian.restype = None
        L.ma2_local_root.argtypes = [_DP, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.ma2_local_root.restype = ctypes.c_double
        L.ma2_sweep.argtypes = [ctypes.c_int, _DP, _DP, ctypes.c_int]
        L.ma2_sweep.restype = ctypes.c_long
        L.ma2_residual.argtypes = [ctypes.c_int, _DP, _DP, _DP]
        L.ma2_residual.restype = ctypes.c_double
        L.ma2_restrict.argtypes = [ctypes.c_int, _DP, _DP, _DP, _DP, ctypes.c_int, ctypes.c_int]
        L.ma2_restrict.restype = None
        L.ma2_prolong_correct.argtypes = [ctypes.c_int, _DP, _DP, _DP]
        L.ma2_prolong_correct.restype = None
        L.ma2_inject.argtypes = [ctypes.c_int, _DP, _DP]
        L.ma2_inject.restype = None
        L.ma2_fmg_interp.argtypes = [ctypes.c_int, _DP, _DP]
        L.ma2_fmg_interp.restype = None
        L.ma2_vcycle.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(Params)]
        L.ma2_vcycle.restype = ctypes.c_long
        L.ma2_fmg.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(Params)]
        L.ma2_fmg.restype = ctypes.c_long
        L.ma2_solve.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(Params),
                                ctypes.POINTER(Report)]
        _ready = True
    return L


def _ptr(a):
    if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
        raise TypeError("oracle arrays must be C-contiguous float64")
    return a.ctypes.data_as(_DP)


def _n(a):
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("2D grid arrays are (n+1, n+1)")
    return a.shape[0] - 1


def params(nu1=2, nu2=2, nu0=1, order="4c", rmode=1, max_cycles=100, tol=1e-10,
           init="fmg") -> Params:
    return Params(nu1, nu2, nu0, ORDERS[order] if isinstance(order, str) else int(order),
                  int(rmode), max_cycles, tol, 2 if init == "fmg" else 0)


def levels(n):
    buf = (ctypes.c_int * 32)()
    k = lib().ma2_levels(n, buf, 32)
    return [buf[i] for i in range(k)]


def hessian(u, i, j):
    g = np.zeros(3)
    lib().ma2_hessian(_n(u), _ptr(u), i, j, _ptr(g))
    return g


def local_root(g, F):
    g = np.ascontiguousarray(g, dtype=np.float64)
    nc = ctypes.c_int(0)
    r = lib().ma2_local_root(_ptr(g), float(F), ctypes.byref(nc))
    return r, bool(nc.value)


def sweep(u, F, order="4c"):
    return lib().ma2_sweep(_n(u), _ptr(u), _ptr(F), ORDERS[order])


def residual(u, F):
    r = np.zeros_like(u)
    ss = lib().ma2_residual(_n(u), _ptr(u), _ptr(F), _ptr(r))
    return r, ss


def restrict(uf, rf, op="ma", rmode=1):
    nc = _n(uf) // 2
    wc = np.zeros((nc + 1, nc + 1))
    bc = np.zeros((nc + 1, nc + 1))
    lib().ma2_restrict(_n(uf), _ptr(uf), _ptr(rf), _ptr(wc), _ptr(bc), 0 if op == "ma" else 1,
                       int(rmode))
    return wc, bc


def prolong_correct(uf, uc, wc):
    lib().ma2_prolong_correct(_n(uf), _ptr(uf), _ptr(uc), _ptr(wc))


def inject(vf):
    vc = np.empty((_n(vf) // 2 + 1,) * 2)
    lib().ma2_inject(_n(vf), _ptr(vf), _ptr(vc))
    return vc


def fmg_interp(uc, uf):
    lib().ma2_fmg_interp(_n(uc), _ptr(uc), _ptr(uf))


def vcycle(u, f, p=None):
    return lib().ma2_vcycle(_n(u), _ptr(u), _ptr(f), ctypes.byref(p or params()))


def fmg(u, f, p=None):
    return lib().ma2_fmg(_n(u), _ptr(u), _ptr(f), ctypes.byref(p or params()))


def solve(u, f, p=None):
    rep = Report()
    st = lib().ma2_solve(_n(u), _ptr(u), _ptr(f), ctypes.byref(p or params()), ctypes.byref(rep))
    if st < 0:
        raise MemoryError("oracle allocation failed")
    return st, rep
