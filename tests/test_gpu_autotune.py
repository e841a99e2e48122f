"""The autotuner on a small mixed batch: it leaves every solver on one of
the candidates it timed (the fastest in its table), and a solve with the
chosen launch shape is bitwise the same as one with the default shape (the
knobs change only how the work is cut into launches)."""
import sys

import numpy as np
import pytest

from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_tune_picks_a_listed_candidate_and_keeps_results():
    from paper_1411_7018_amd import Solver, autotune
    from paper_1411_7018_amd.batch import solve_batch
    specs = [("exp_cos", 32, 11), ("quadratic", 48, 12), ("exp_cos", 64, 13)]
    note("autotune", specs)
    data = [P.make_device(k, n, sd) for k, n, sd in specs]
    solvers = [Solver(n) for _, n, _ in specs]
    cand = dict(blocks=(4096, 65536), coarse=(0, 16), strips=(8, 128), block_ns=(-1, 64),
                tiles=(0, 2), zsweeps=(0, 32))
    ch = autotune.tune(solvers, [d[0] for d in data], [d[1] for d in data], ticks=2, **cand)
    assert ch.coarse_n in cand["coarse"] and ch.max_blocks in cand["blocks"]
    assert ch.strip_rows in cand["strips"] + (0,) and ch.block_n in cand["block_ns"] + (0,)
    assert ch.tile_config in cand["tiles"] and ch.zsweep_n in cand["zsweeps"]
    best = min(ch.table, key=lambda r: r[-1])
    assert (ch.coarse_n, ch.max_blocks, ch.strip_rows, ch.block_n, ch.tile_config,
            ch.zsweep_n) == tuple(best[:6])
    for s in solvers:
        p = s.params
        assert (p.coarse_n, p.max_blocks, p.strip_rows, p.block_n, p.tile_config,
                p.zsweep_n) == tuple(best[:6])
    tuned = [d[0].clone() for d in data]
    st, reps = solve_batch(solvers, tuned, [d[1] for d in data], tol=1e-8)
    assert st == 0
    plain = [d[0].clone() for d in data]
    st2, reps2 = solve_batch([Solver(n) for _, n, _ in specs], plain, [d[1] for d in data],
                             tol=1e-8)
    assert st2 == 0
    for a, b, ra, rb in zip(tuned, plain, reps, reps2):
        assert ra["cycles"] == rb["cycles"]
        assert torch.equal(a, b)


def test_every_smoother_shape_same_bits():
    """Each tile_config and z-stream setting, forced on a 64^3 solve, gives
    the default solve's result bit for bit."""
    from paper_1411_7018_amd import Solver
    n = 64
    u0, f = P.make_device("exp_cos", n, 21)
    ref = u0.clone()
    Solver(n).solve(ref, f, tol=1e-8)
    for tc, zn in ((1, 0), (2, 0), (4, 0), (6, 0), (7, 0), (0, 64), (8, 64), (9, 32),
                   (10, 64), (11, 32), (0, -1)):
        note("shape", tc, zn)
        u = u0.clone()
        Solver(n, tile_config=tc, zsweep_n=zn).solve(u, f, tol=1e-8)
        assert torch.equal(u, ref), (tc, zn)
