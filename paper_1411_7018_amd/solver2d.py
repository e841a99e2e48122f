"""Solver2D: a torch-facing handle over one ma2d_solver (include/ma2d.h), the
two-dimensional variant u_xx u_yy - u_xy^2 = f.  Grid functions are
contiguous float64 CUDA (HIP) tensors of shape (n+1, n+1) indexed [j, i]
(x fastest); every computation runs in libmafas.so.
"""
from __future__ import annotations

import torch

from . import _lib as L

_ORDERS = {"rb": L.MA2D_RED_BLACK, "red_black": L.MA2D_RED_BLACK, "4c": L.MA2D_COLOR4}
_RESTRICT = {"full": L.MA_RESTRICT_FULL, "half": L.MA_RESTRICT_HALF}


class Solver2D:
    def __init__(self, n: int, stream=None, **params):
        self.n = int(n)
        p = L.ma2d_params_default(self.n)
        for k, v in params.items():
            if k == "order" and isinstance(v, str):
                v = _ORDERS[v]
            if k == "restriction" and isinstance(v, str):
                v = _RESTRICT[v]
            setattr(p, k, v)
        self.params = p
        if stream is None:
            stream = torch.cuda.current_stream()
        self._h = None
        self._h = L.ma2d_create(p, stream.cuda_stream or None)

    def close(self):
        if self._h:
            L.ma2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _g(self, t, name="u") -> int:
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if tuple(t.shape) != (self.n + 1,) * 2 or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {(self.n + 1,) * 2}")
        return t.data_ptr()

    def sweep(self, u, f, count: int = 1) -> int:
        return L.ma2d_sweep(self._h, self._g(u), self._g(f, "f"), count)

    def residual(self, u, f, out=None) -> float:
        return L.ma2d_residual(self._h, self._g(u), self._g(f, "f"),
                               self._g(out, "out") if out is not None else None)

    def vcycle(self, u, f) -> None:
        L.ma2d_vcycle(self._h, self._g(u), self._g(f, "f"))

    def fmg(self, u, f) -> int:
        return L.ma2d_fmg(self._h, self._g(u), self._g(f, "f"))

    def solve(self, u, f, tol: float | None = None, init: str = "fmg") -> dict:
        flags = L.MA_INIT_FMG if init == "fmg" else 0
        return L.ma2d_solve(self._h, self._g(u), self._g(f, "f"),
                            tol if tol is not None else -1.0, flags).as_dict()
