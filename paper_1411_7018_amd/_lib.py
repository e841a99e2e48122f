"""ctypes binding of the C ABI in include/ma.h (argument marshalling only).

Every function here has the name of the C entry point it calls; all the
arithmetic happens in libmafas.so's HIP kernels.  The library is loaded from
the package directory and must have been built (``__graft_entry__.build()`` or
``python -m paper_1411_7018_amd.build``); a missing library raises at import of
this module, with no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmafas.so")

MA_OK, MA_ERR_ARG, MA_ERR_OOM, MA_ERR_DEVICE, MA_ERR_NOT_CONVERGED, MA_ERR_NONFINITE = range(6)
MA_FP64, MA_MIXED = 0, 1
MA_COLOR4, MA_COLOR8 = 0, 1
MA_RESTRICT_FULL, MA_RESTRICT_HALF = 0, 1
MA_SMOOTHER_AUTO, MA_SMOOTHER_COLOR, MA_SMOOTHER_FUSED = 0, 1, 2
MA_INIT_POISSON = 1
MA_INIT_FMG = 2

STATUS_NAMES = {0: "MA_OK", 1: "MA_ERR_ARG", 2: "MA_ERR_OOM", 3: "MA_ERR_DEVICE",
                4: "MA_ERR_NOT_CONVERGED", 5: "MA_ERR_NONFINITE"}


class ma_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("nu0", ctypes.c_int), ("order", ctypes.c_int), ("restriction", ctypes.c_int),
                ("precision", ctypes.c_int), ("smoother", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("tol", ctypes.c_double),
                ("init_tol", ctypes.c_double), ("init_max_cycles", ctypes.c_int),
                ("inner_cycles", ctypes.c_int), ("profile", ctypes.c_int),
                ("tile_config", ctypes.c_int), ("block_n", ctypes.c_int),
                ("graphs", ctypes.c_int), ("coarse_n", ctypes.c_int),
                ("max_blocks", ctypes.c_int), ("strip_rows", ctypes.c_int),
                ("zsweep_n", ctypes.c_int), ("fuse_prolong", ctypes.c_int)]


class ma2d_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("nu0", ctypes.c_int), ("order", ctypes.c_int), ("restriction", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("tol", ctypes.c_double)]


MA2D_COLOR4, MA2D_RED_BLACK = 0, 1


class ma_report(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("outer", ctypes.c_int), ("init_cycles", ctypes.c_int),
                ("converged", ctypes.c_int), ("res0", ctypes.c_double), ("res", ctypes.c_double),
                ("rel_res", ctypes.c_double), ("nonconvex", ctypes.c_longlong),
                ("fp64_fallbacks", ctypes.c_longlong), ("seconds", ctypes.c_double),
                ("point_updates", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("history", ctypes.c_double * 64), ("smooth_launches", ctypes.c_int),
                ("smooth_seconds", ctypes.c_double), ("smooth_bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "history"}
        d["history"] = [self.history[i] for i in range(min(self.cycles, 64))]
        return d


class MAError(RuntimeError):
    def __init__(self, status: int, message: str, report: dict | None = None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.report = report


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python -m paper_1411_7018_amd.build)")

_L = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_P = ctypes.POINTER(ma_params)
_R = ctypes.POINTER(ma_report)

_L.ma_params_default.argtypes = [_P, ctypes.c_int]
_L.ma_params_default.restype = None
_L.ma_footprint_bytes.argtypes = [_P]
_L.ma_footprint_bytes.restype = ctypes.c_size_t
_L.ma_levels.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
_L.ma_levels.restype = ctypes.c_int
_L.ma_create.argtypes = [_P, _vp, ctypes.POINTER(_vp)]
_L.ma_destroy.argtypes = [_vp]
_L.ma_destroy.restype = None
_L.ma_last_error.argtypes = [_vp]
_L.ma_last_error.restype = ctypes.c_char_p
_L.ma_set_stream.argtypes = [_vp, _vp]
_L.ma_retune.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
_L.ma_retune_smoother.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
_L.ma_residual_noalloc.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp]
_L.ma_residual_noalloc.restype = ctypes.c_int
_L.ma_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_uint, _R]
_L.ma_vcycle.argtypes = [_vp, _vp, _vp]
_L.ma_residual.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
_L.ma_sweep.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
_L.ma_restrict.argtypes = [_vp, _vp, _vp, _vp, _vp]
_L.ma_prolong_correct.argtypes = [_vp, _vp, _vp, _vp]
_L.ma_poisson_init.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int)]
_L.ma_fmg.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_longlong)]
_L.ma_gs_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _R]
_L.ma_solve_batch.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                              ctypes.c_int, ctypes.c_double, ctypes.c_uint, _R]
_L.ma_batch_create.argtypes = [ctypes.c_int, _vp, ctypes.POINTER(_vp)]
_L.ma_batch_destroy.argtypes = [_vp]
_L.ma_batch_destroy.restype = None
_L.ma_batch_last_error.argtypes = [_vp]
_L.ma_batch_last_error.restype = ctypes.c_char_p
_L.ma_batch_add.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_uint,
                            ctypes.POINTER(ctypes.c_int)]
_L.ma_batch_tick.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
_L.ma_batch_report.argtypes = [_vp, ctypes.c_int, _R]
_L.ma_batch_remove.argtypes = [_vp, ctypes.c_int]
_P2 = ctypes.POINTER(ma2d_params)
_L.ma2d_params_default.argtypes = [_P2, ctypes.c_int]
_L.ma2d_params_default.restype = None
_L.ma2d_footprint_bytes.argtypes = [_P2]
_L.ma2d_footprint_bytes.restype = ctypes.c_size_t
_L.ma2d_create.argtypes = [_P2, _vp, ctypes.POINTER(_vp)]
_L.ma2d_destroy.argtypes = [_vp]
_L.ma2d_destroy.restype = None
_L.ma2d_last_error.argtypes = [_vp]
_L.ma2d_last_error.restype = ctypes.c_char_p
_L.ma2d_sweep.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
_L.ma2d_residual.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
_L.ma2d_vcycle.argtypes = [_vp, _vp, _vp]
_L.ma2d_fmg.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_longlong)]
_L.ma2d_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_uint, _R]
for _name in ("ma2d_create", "ma2d_sweep", "ma2d_residual", "ma2d_vcycle", "ma2d_fmg",
              "ma2d_solve"):
    getattr(_L, _name).restype = ctypes.c_int
for _name in ("ma_create", "ma_set_stream", "ma_retune", "ma_retune_smoother", "ma_solve",
              "ma_vcycle",
              "ma_residual", "ma_sweep", "ma_restrict", "ma_prolong_correct", "ma_poisson_init",
              "ma_fmg", "ma_gs_solve", "ma_solve_batch", "ma_batch_create", "ma_batch_add",
              "ma_batch_tick",
              "ma_batch_report", "ma_batch_remove"):
    getattr(_L, _name).restype = ctypes.c_int

EXPORTS = ("ma_params_default", "ma_footprint_bytes", "ma_levels", "ma_create", "ma_destroy",
           "ma_last_error", "ma_set_stream", "ma_retune", "ma_retune_smoother", "ma_solve",
           "ma_vcycle",
           "ma_residual", "ma_residual_noalloc", "ma_sweep", "ma_restrict",
           "ma_prolong_correct", "ma_poisson_init",
           "ma_fmg", "ma_gs_solve", "ma_solve_batch", "ma_batch_create", "ma_batch_destroy",
           "ma_batch_last_error", "ma_batch_add", "ma_batch_tick", "ma_batch_report",
           "ma_batch_remove", "ma2d_params_default", "ma2d_footprint_bytes", "ma2d_create",
           "ma2d_destroy", "ma2d_last_error", "ma2d_sweep", "ma2d_residual", "ma2d_vcycle",
           "ma2d_fmg", "ma2d_solve")


def lib() -> ctypes.CDLL:
    return _L


def _check(st: int, handle=None, batch=None):
    if st != MA_OK:
        if batch is not None:
            msg = _L.ma_batch_last_error(batch)
        else:
            msg = _L.ma_last_error(handle)
        raise MAError(st, (msg or b"").decode())


def ma_params_default(n: int) -> ma_params:
    p = ma_params()
    _L.ma_params_default(ctypes.byref(p), int(n))
    return p


def ma_footprint_bytes(p: ma_params) -> int:
    return int(_L.ma_footprint_bytes(ctypes.byref(p)))


def ma_levels(n: int) -> list[int]:
    buf = (ctypes.c_int * 32)()
    L = _L.ma_levels(int(n), buf, 32)
    return [buf[i] for i in range(L)]


def ma_create(p: ma_params, stream: int | None) -> int:
    h = _vp()
    _check(_L.ma_create(ctypes.byref(p), stream or None, ctypes.byref(h)), None)
    return h.value


def ma_destroy(h: int) -> None:
    _L.ma_destroy(h)


def ma_last_error(h: int | None) -> str:
    return (_L.ma_last_error(h) or b"").decode()


def ma_set_stream(h: int, stream: int | None) -> None:
    _check(_L.ma_set_stream(h, stream or None), h)


def ma_retune(h: int, coarse_n: int, max_blocks: int, strip_rows: int, block_n: int = 0) -> None:
    _check(_L.ma_retune(h, int(coarse_n), int(max_blocks), int(strip_rows), int(block_n)), h)


def ma_residual_noalloc(n: int, u: int, f: int, r: int | None, l2_dev: int, stream) -> None:
    """The allocation-free residual (device pointers as integers; the norm
    lands in the device double at l2_dev)."""
    st = _L.ma_residual_noalloc(int(n), u, f, r or None, l2_dev, stream or None)
    if st != MA_OK:
        raise MAError(st, ma_last_error(None))


def ma_retune_smoother(h: int, block_n: int, zsweep_n: int, tile_config: int) -> None:
    _check(_L.ma_retune_smoother(h, int(block_n), int(zsweep_n), int(tile_config)), h)


def ma_solve(h: int, u: int, f: int, tol: float, flags: int) -> ma_report:
    rep = ma_report()
    st = _L.ma_solve(h, u, f, float(tol), int(flags), ctypes.byref(rep))
    if st != MA_OK:
        raise MAError(st, ma_last_error(h), rep.as_dict())
    return rep


def ma_vcycle(h: int, u: int, f: int) -> None:
    _check(_L.ma_vcycle(h, u, f), h)


def ma_residual(h: int, u: int, f: int, r: int | None) -> float:
    out = ctypes.c_double()
    _check(_L.ma_residual(h, u, f, r or None, ctypes.byref(out)), h)
    return out.value


def ma_sweep(h: int, u: int, f: int, count: int) -> int:
    nc = ctypes.c_longlong()
    _check(_L.ma_sweep(h, u, f, int(count), ctypes.byref(nc)), h)
    return nc.value


def ma_restrict(h: int, u: int, f: int, w_c: int, b_c: int) -> None:
    _check(_L.ma_restrict(h, u, f, w_c, b_c), h)


def ma_prolong_correct(h: int, u: int, u_c: int, w_c: int) -> None:
    _check(_L.ma_prolong_correct(h, u, u_c, w_c), h)


def ma_poisson_init(h: int, u: int, f: int) -> int:
    c = ctypes.c_int()
    _check(_L.ma_poisson_init(h, u, f, ctypes.byref(c)), h)
    return c.value


def ma_fmg(h: int, u: int, f: int) -> int:
    nc = ctypes.c_longlong()
    _check(_L.ma_fmg(h, u, f, ctypes.byref(nc)), h)
    return nc.value


def ma_gs_solve(h: int, u: int, f: int, tol: float, max_sweeps: int) -> ma_report:
    rep = ma_report()
    st = _L.ma_gs_solve(h, u, f, float(tol), int(max_sweeps), ctypes.byref(rep))
    if st != MA_OK:
        raise MAError(st, ma_last_error(h), rep.as_dict())
    return rep


def ma_solve_batch(handles, us, fs, tol: float, flags: int):
    n = len(handles)
    H = (_vp * n)(*handles)
    U = (_vp * n)(*us)
    F = (_vp * n)(*fs)
    reps = (ma_report * n)()
    st = _L.ma_solve_batch(H, U, F, n, float(tol), int(flags), reps)
    return st, [reps[i] for i in range(n)]


def ma_batch_create(max_solves: int, stream: int | None) -> int:
    b = _vp()
    st = _L.ma_batch_create(int(max_solves), stream or None, ctypes.byref(b))
    if st != MA_OK:
        raise MAError(st, "ma_batch_create failed")
    return b.value


def ma_batch_destroy(b: int) -> None:
    _L.ma_batch_destroy(b)


def ma_batch_add(b: int, h: int, u: int, f: int, tol: float, flags: int) -> int:
    slot = ctypes.c_int()
    _check(_L.ma_batch_add(b, h, u, f, float(tol), int(flags), ctypes.byref(slot)), batch=b)
    return slot.value


def ma_batch_tick(b: int, max_solves: int):
    done = (ctypes.c_int * max_solves)()
    st = _L.ma_batch_tick(b, done)
    return st, [done[i] for i in range(max_solves)]


def ma_batch_report(b: int, slot: int) -> ma_report:
    rep = ma_report()
    _check(_L.ma_batch_report(b, int(slot), ctypes.byref(rep)), batch=b)
    return rep


def ma_batch_remove(b: int, slot: int) -> None:
    _check(_L.ma_batch_remove(b, int(slot)), batch=b)


# ---------------------------------------------------------------------------
# 2D variant (include/ma2d.h)
# ---------------------------------------------------------------------------
def _check2(st: int, h=None):
    if st != MA_OK:
        raise MAError(st, (_L.ma2d_last_error(h) or b"").decode())


def ma2d_params_default(n: int) -> ma2d_params:
    p = ma2d_params()
    _L.ma2d_params_default(ctypes.byref(p), int(n))
    return p


def ma2d_footprint_bytes(p: ma2d_params) -> int:
    return _L.ma2d_footprint_bytes(ctypes.byref(p))


def ma2d_create(p: ma2d_params, stream: int | None) -> int:
    h = _vp()
    _check2(_L.ma2d_create(ctypes.byref(p), stream or None, ctypes.byref(h)))
    return h.value


def ma2d_destroy(h: int) -> None:
    _L.ma2d_destroy(h)


def ma2d_sweep(h: int, u: int, f: int, count: int) -> int:
    nc = ctypes.c_longlong()
    _check2(_L.ma2d_sweep(h, u, f, int(count), ctypes.byref(nc)), h)
    return nc.value


def ma2d_residual(h: int, u: int, f: int, r: int | None) -> float:
    out = ctypes.c_double()
    _check2(_L.ma2d_residual(h, u, f, r or None, ctypes.byref(out)), h)
    return out.value


def ma2d_vcycle(h: int, u: int, f: int) -> None:
    _check2(_L.ma2d_vcycle(h, u, f), h)


def ma2d_fmg(h: int, u: int, f: int) -> int:
    nc = ctypes.c_longlong()
    _check2(_L.ma2d_fmg(h, u, f, ctypes.byref(nc)), h)
    return nc.value


def ma2d_solve(h: int, u: int, f: int, tol: float, flags: int) -> ma_report:
    rep = ma_report()
    st = _L.ma2d_solve(h, u, f, float(tol), int(flags), ctypes.byref(rep))
    if st != MA_OK:
        raise MAError(st, (_L.ma2d_last_error(h) or b"").decode(), rep.as_dict())
    return rep
