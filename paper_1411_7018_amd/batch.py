"""Batched solves over the C ABI (ma_solve_batch, ma_batch_*).

A batch advances many independent Monge-Ampere solves of different grid
sizes together: every level phase of every V-cycle is one launch for all of
them (see the engine in csrc/ma_engine.hip).  ``solve_batch`` solves a fixed
set to completion; ``ResidentBatch`` keeps a slot table for continuous
serving, where solves join and leave between ticks.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .solver import Solver


def _flags(init_poisson, init):
    if init is None:
        init = "poisson" if init_poisson else "none"
    return {"poisson": L.MA_INIT_POISSON, "fmg": L.MA_INIT_FMG, "none": 0}[init]


def solve_batch(solvers, us, fs, tol: float | None = None, init_poisson: bool = True,
                init: str | None = None):
    """Solve len(solvers) problems together; returns (status, [report dict]).
    init: "poisson" (default), "fmg" or "none"."""
    if not (len(solvers) == len(us) == len(fs)):
        raise ValueError("solvers, us and fs must have the same length")
    hs, up, fp = [], [], []
    for s, u, f in zip(solvers, us, fs):
        hs.append(s.handle)
        up.append(s._grid(u))
        fp.append(s._grid(f, name="f"))
    flags = _flags(init_poisson, init)
    st, reps = L.ma_solve_batch(hs, up, fp, tol if tol is not None else -1.0, flags)
    return st, [r.as_dict() for r in reps]


class ResidentBatch:
    """Slot table of a resident batch (at most 64 concurrent solves)."""

    def __init__(self, max_solves: int = 64, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        self.max_solves = int(max_solves)
        self._b = L.ma_batch_create(self.max_solves, stream.cuda_stream or None)
        self._refs = {}

    def close(self):
        if self._b:
            L.ma_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, solver: Solver, u, f, tol: float | None = None, init_poisson=True,
            init: str | None = None) -> int:
        """Join a solve; init: "poisson" (default), "fmg" (its FMG-FAS
        iteration runs now, synchronously) or "none"."""
        flags = _flags(init_poisson, init)
        slot = L.ma_batch_add(self._b, solver.handle, solver._grid(u), solver._grid(f, name="f"),
                              tol if tol is not None else -1.0, flags)
        self._refs[slot] = (solver, u, f)   # keep the tensors alive while resident
        return slot

    def tick(self):
        """One step of every resident solve; returns {slot: 1 converged, 2 failed}
        for the slots that finished in this tick."""
        st, done = L.ma_batch_tick(self._b, self.max_solves)
        if st != L.MA_OK:
            raise L.MAError(st, (L.lib().ma_batch_last_error(self._b) or b"").decode())
        return {i: d for i, d in enumerate(done) if d}

    def report(self, slot: int) -> dict:
        return L.ma_batch_report(self._b, slot).as_dict()

    def remove(self, slot: int) -> None:
        L.ma_batch_remove(self._b, slot)
        self._refs.pop(slot, None)

    @property
    def active(self) -> int:
        return len(self._refs)
