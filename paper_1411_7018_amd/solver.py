"""Solver: a torch-facing handle over one ma_solver (include/ma.h).

Tensors are only marshalled: every computation runs in libmafas.so.  Grid
functions are contiguous float64 CUDA (HIP) tensors of shape (n+1, n+1, n+1)
indexed [k, j, i], i.e. x fastest, as the C ABI requires.
"""
from __future__ import annotations

import torch

from . import _lib as L

_ORDERS = {"4c": L.MA_COLOR4, "color4": L.MA_COLOR4, "8c": L.MA_COLOR8, "color8": L.MA_COLOR8}
_PREC = {"fp64": L.MA_FP64, "mixed": L.MA_MIXED}
_RESTRICT = {"full": L.MA_RESTRICT_FULL, "half": L.MA_RESTRICT_HALF}
_SMOOTHER = {"auto": L.MA_SMOOTHER_AUTO, "color": L.MA_SMOOTHER_COLOR,
             "fused": L.MA_SMOOTHER_FUSED}


def make_params(n: int, **kw) -> L.ma_params:
    p = L.ma_params_default(n)
    for key, val in kw.items():
        if val is None:
            continue
        if key == "order":
            val = _ORDERS[val] if isinstance(val, str) else int(val)
        elif key == "precision":
            val = _PREC[val] if isinstance(val, str) else int(val)
        elif key == "restriction":
            val = _RESTRICT[val] if isinstance(val, str) else int(val)
        elif key == "smoother":
            val = _SMOOTHER[val] if isinstance(val, str) else int(val)
        setattr(p, key, val)
    return p


def footprint_bytes(n: int, **kw) -> int:
    return L.ma_footprint_bytes(make_params(n, **kw))


def _stream_handle(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


class Solver:
    """One resident multigrid hierarchy for (n+1)^3 problems."""

    def __init__(self, n: int, stream=None, **params):
        self.n = int(n)
        self.params = make_params(self.n, **params)
        self._h = None
        self._h = L.ma_create(self.params, _stream_handle(stream))

    def close(self):
        if self._h:
            L.ma_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> int:
        if not self._h:
            raise RuntimeError("solver is closed")
        return self._h

    def set_stream(self, stream) -> None:
        L.ma_set_stream(self.handle, _stream_handle(stream))

    def retune(self, coarse_n: int | None = None, max_blocks: int | None = None,
               strip_rows: int | None = None, block_n: int | None = None,
               zsweep_n: int | None = None, tile_config: int | None = None) -> None:
        """Change the launch shape of later cycles (results are unchanged)."""
        cn = self.params.coarse_n if coarse_n is None else int(coarse_n)
        mb = self.params.max_blocks if max_blocks is None else int(max_blocks)
        sr = self.params.strip_rows if strip_rows is None else int(strip_rows)
        bn = self.params.block_n if block_n is None else int(block_n)
        zn = self.params.zsweep_n if zsweep_n is None else int(zsweep_n)
        tc = self.params.tile_config if tile_config is None else int(tile_config)
        L.ma_retune(self.handle, cn, mb, sr, bn)
        L.ma_retune_smoother(self.handle, bn, zn, tc)
        p = self.params
        p.coarse_n, p.max_blocks, p.strip_rows, p.block_n = cn, mb, sr, bn
        p.zsweep_n, p.tile_config = zn, tc

    def _grid(self, t: torch.Tensor, n: int | None = None, name: str = "u") -> int:
        n = self.n if n is None else n
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if tuple(t.shape) != (n + 1,) * 3 or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {(n + 1,) * 3}")
        return t.data_ptr()

    def solve(self, u, f, tol: float | None = None, init_poisson: bool = True,
              init: str | None = None) -> dict:
        """init: "poisson" (default), "fmg" (Section 4 protocol: one FMG-FAS
        iteration as the first cycle) or "none"; init_poisson=False is the
        same as init="none"."""
        if init is None:
            init = "poisson" if init_poisson else "none"
        flags = {"poisson": L.MA_INIT_POISSON, "fmg": L.MA_INIT_FMG, "none": 0}[init]
        rep = L.ma_solve(self.handle, self._grid(u), self._grid(f, name="f"),
                         tol if tol is not None else -1.0, flags)
        return rep.as_dict()

    def vcycle(self, u, f) -> None:
        L.ma_vcycle(self.handle, self._grid(u), self._grid(f, name="f"))

    def residual(self, u, f, out=None) -> float:
        r = self._grid(out, name="out") if out is not None else None
        return L.ma_residual(self.handle, self._grid(u), self._grid(f, name="f"), r)

    def sweep(self, u, f, count: int = 1) -> int:
        return L.ma_sweep(self.handle, self._grid(u), self._grid(f, name="f"), count)

    def restrict(self, u, f):
        nc = self.n // 2
        w = torch.empty((nc + 1,) * 3, dtype=torch.float64, device=u.device)
        b = torch.empty_like(w)
        L.ma_restrict(self.handle, self._grid(u), self._grid(f, name="f"), w.data_ptr(),
                      b.data_ptr())
        return w, b

    def prolong_correct(self, u, uc, wc) -> None:
        nc = self.n // 2
        L.ma_prolong_correct(self.handle, self._grid(u), self._grid(uc, nc, "uc"),
                             self._grid(wc, nc, "wc"))

    def gs_solve(self, u, f, tol: float | None = None, max_sweeps: int = 100000) -> dict:
        """The standalone nonlinear Gauss-Seidel solver (no multigrid)."""
        rep = L.ma_gs_solve(self.handle, self._grid(u), self._grid(f, name="f"),
                            tol if tol is not None else -1.0, max_sweeps)
        return rep.as_dict()

    def fmg(self, u, f) -> int:
        """One FMG-FAS iteration (Algorithm 2); returns non-certified updates."""
        return L.ma_fmg(self.handle, self._grid(u), self._grid(f, name="f"))

    def poisson_init(self, u, f) -> int:
        return L.ma_poisson_init(self.handle, self._grid(u), self._grid(f, name="f"))


def levels(n: int) -> list[int]:
    return L.ma_levels(n)
