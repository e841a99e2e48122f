"""Autotuner for the launch shapes of the batched engine.

The engine's arithmetic is fixed; what changes its speed is how the work is
cut into launches:
  * ``max_blocks`` -- the cap on the blocks of one row-kernel launch.  Few
    blocks walk many rows each inside one XCD's window (good L2 reuse of the
    stencil halos on big grids); many blocks put more waves in flight (good
    latency hiding).  The largest caps give the 385^3 finest level one row
    per block.
  * ``coarse_n``   -- levels with n <= coarse_n run inside the
    single-workgroup coarse-level kernel instead of one launch per phase.
  * ``strip_rows`` -- the width of the y-strips in which a launch walks its
    rows along z: narrow strips keep the planes a stencil re-reads in L2.
  * ``block_n``    -- levels with n <= block_n (above coarse_n) smooth with
    block sweeps (the four colour phases of a sweep in one launch) instead
    of one launch per colour phase; -1 turns them off.
  * ``tile_config`` -- the block shape of those block sweeps (0: picked by
    the level's size and block count; 1..7 fixed shapes).
  * ``zsweep_n``   -- levels with n >= zsweep_n smooth with z-stream sweeps
    (four colour phases per launch, each workgroup walking a column plane by
    plane); 0 automatic, -1 never.

``tune`` times the candidates on the device, on the caller's own
solvers and data (a copy of u), with one tick per candidate for graph
capture followed by timed ticks, and leaves the solvers retuned to the
fastest pair.  All candidates give bitwise the same results, so tuning never
changes what a solve computes.  ``load`` / ``save`` keep choices in a JSON
file keyed by device name, grid sizes and precision.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import torch

BLOCKS = (4096, 8192, 16384, 32768, 65536, 131072, 262144)
COARSE = (0, 8, 16, 32)
STRIPS = (8, 32, 128, 4096)
BLOCK_N = (-1, 32, 64)
TILES = (0, 1, 2, 5, 6)
ZSWEEP = (0, -1)


@dataclasses.dataclass
class Choice:
    coarse_n: int
    max_blocks: int
    strip_rows: int
    block_n: int
    seconds_per_tick: float
    # [(coarse_n, max_blocks, strip_rows, block_n, tile_config, zsweep_n, seconds_per_tick)]
    table: list
    tile_config: int = 0
    zsweep_n: int = 0

    def as_dict(self) -> dict:
        return {"coarse_n": self.coarse_n, "max_blocks": self.max_blocks,
                "strip_rows": self.strip_rows, "block_n": self.block_n,
                "tile_config": self.tile_config, "zsweep_n": self.zsweep_n,
                "seconds_per_tick": self.seconds_per_tick,
                "table": [list(r) for r in self.table]}


def key(sizes, precision: str, order: str = "4c") -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{dev}|{precision}|{order}|" + ",".join(str(n) for n in sorted(sizes))


def _time_ticks(solvers, us, fs, ticks: int) -> float:
    from .batch import ResidentBatch

    b = ResidentBatch(len(solvers))
    try:
        work = [u.clone() for u in us]
        for s, u, f in zip(solvers, work, fs):
            # an unreachable tolerance keeps every solve cycling
            b.add(s, u, f, tol=1e-300, init_poisson=False)
        b.tick()                       # entry residuals, first tick, capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(ticks):
            b.tick()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / ticks
    finally:
        b.close()


def tune(solvers, us, fs, ticks: int = 4, blocks=BLOCKS, coarse=COARSE, strips=STRIPS,
         block_ns=BLOCK_N, tiles=TILES, zsweeps=ZSWEEP, verbose: bool = False) -> Choice:
    """Pick the launch shape of one batched tick of these solves and retune
    the solvers to it.  The knobs barely interact (coarse_n moves work
    between the coarse-level kernel and the row kernels; max_blocks and
    strip_rows shape the row kernels; block_n and tile_config move and shape
    the mid-level block sweeps; zsweep_n moves the largest levels to the
    z-stream sweep), so they are searched one after the other -- coarse_n x
    max_blocks on the default strips, then strip_rows, then block_n, then
    tile_config, then zsweep_n -- instead of over the full product.  The
    solves must fit one batch (at most 64, shared smoothing parameters)."""
    if not solvers:
        raise ValueError("nothing to tune")
    if any(s.params.max_cycles < ticks + 1 for s in solvers):
        raise ValueError("max_cycles must exceed the number of timed ticks")
    # time from where a solve's FAS cycles start: after the Poisson guess
    starts = []
    for s, u, f in zip(solvers, us, fs):
        w = u.clone()
        s.poisson_init(w, f)
        starts.append(w)
    table = []

    def trial(cn, mb, sr, bn, tc=0, zn=0):
        for s in solvers:
            s.retune(coarse_n=cn, max_blocks=mb, strip_rows=sr, block_n=bn, tile_config=tc,
                     zsweep_n=zn)
        t = min(_time_ticks(solvers, starts, fs, ticks) for _ in range(2))
        table.append((cn, mb, sr, bn, tc, zn, t))
        if verbose:
            print(f"[tune] coarse_n={cn:2d} max_blocks={mb:6d} strip_rows={sr:4d} "
                  f"block_n={bn:4d} tile_config={tc:2d} zsweep_n={zn:3d}: "
                  f"{1e3 * t:.3f} ms/tick", flush=True)
        return t

    def best():
        return min(table, key=lambda r: r[6])

    for cn in coarse:
        for mb in blocks:
            trial(cn, mb, 0, 0)
    cn, mb, _, _, _, _, _ = best()
    for sr in strips:
        trial(cn, mb, sr, 0)
    cn, mb, sr, _, _, _, _ = best()
    for bn in block_ns:
        trial(cn, mb, sr, bn)
    cn, mb, sr, bn, _, _, _ = best()
    if bn != -1:
        for tc in tiles:
            trial(cn, mb, sr, bn, tc)
    cn, mb, sr, bn, tc, _, _ = best()
    for zn in zsweeps:
        trial(cn, mb, sr, bn, tc, zn)
    cn, mb, sr, bn, tc, zn, t = best()
    for s in solvers:
        s.retune(coarse_n=cn, max_blocks=mb, strip_rows=sr, block_n=bn, tile_config=tc,
                 zsweep_n=zn)
    return Choice(cn, mb, sr, bn, t, table, tc, zn)


def load(path: str, k: str) -> dict | None:
    try:
        with open(path) as fh:
            return json.load(fh).get(k)
    except (OSError, ValueError):
        return None


def save(path: str, k: str, choice: Choice) -> None:
    data = {}
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        pass
    data[k] = choice.as_dict()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
