"""Oracle parity of the engine at the benchmark's full sizes and launch
shapes (Algorithm 1; the stopping rule's norm of Section 4).

One FAS V(2,2) cycle at 257^3 and 385^3 runs through the batched engine
exactly as a timed solve runs it -- the finest-level colour phases of
k_batched reading the colour-ordered right-hand side in y-strips, the fused
residual-restriction, the block sweeps of the middle levels, the coarse
levels in one LDS workgroup -- with the launch shapes the autotuner picks
for these sizes, and the same cycle runs in the oracle from the same start.
The start is the exact solution plus a smooth bump that vanishes on the
boundary (0.01 sin(pi x) sin(pi y) sin(pi z), which keeps the Hessian SPD).

Checked: the cycle's result node by node (<= 1e-12 relative max-norm), the
engine's residual norm of the start (its r0) against the oracle's sum of
squares, and the engine's norm after the cycle against the oracle's
residual of the engine's own result.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-12

# (kind, n, seed) -> launch shapes (coarse_n, max_blocks, strip_rows, block_n)
CASES = {
    ("exp_cos", 256, 3001): [(16, 131072, 32, 0), (16, 65536, 128, 0)],
    ("exp_cos", 384, 5001): [(16, 262144, 32, 0), (16, 65536, 8, 0)],
}
_cache = {}


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def start(kind, n, seed):
    """(u_start and f on the device, the oracle's r0 sum of squares and its
    one-cycle result on the host), computed once per problem."""
    key = (kind, n, seed)
    if key not in _cache:
        u0, f, ue = P.make_device(kind, n, seed, exact=True)
        t = torch.arange(n + 1, dtype=torch.float64, device="cuda") / n
        s = torch.sin(math.pi * t)
        bump = 0.01 * s[:, None, None] * s[None, :, None] * s[None, None, :]
        us = ue + bump
        us[0], us[-1] = ue[0], ue[-1]
        us[:, 0], us[:, -1] = ue[:, 0], ue[:, -1]
        us[:, :, 0], us[:, :, -1] = ue[:, :, 0], ue[:, :, -1]
        del u0, ue, bump
        torch.cuda.synchronize()
        uh = us.cpu().numpy()
        fh = f.cpu().numpy()
        _, ss0 = oracle.residual(uh, fh, out=False)
        uo = uh.copy()
        oracle.vcycle(uo, fh)
        del uh
        _cache.clear()
        _cache[key] = (us, f, fh, ss0, uo)
    return _cache[key]


@pytest.mark.parametrize("kind,n,seed,shape",
                         [(k, n, s, sh) for (k, n, s), shapes in CASES.items() for sh in shapes])
def test_engine_cycle_at_bench_shape_matches_oracle(kind, n, seed, shape):
    from paper_1411_7018_amd import Solver, _lib as L
    note("bench-shape cycle", kind, n, "shape", shape)
    us, f, fh, ss0, uo = start(kind, n, seed)
    cn, mb, sr, bn = shape
    s = Solver(n, max_cycles=1, coarse_n=cn, max_blocks=mb, strip_rows=sr, block_n=bn)
    u = us.clone()
    with pytest.raises(L.MAError) as ei:
        s.solve(u, f, tol=1e-300, init="none")
    assert ei.value.status == L.MA_ERR_NOT_CONVERGED
    rep = ei.value.report
    assert rep["cycles"] == 1
    torch.cuda.synchronize()
    ug = u.cpu().numpy()
    # the V-cycle, node by node
    err = np.abs(ug - uo).max() / np.abs(uo).max()
    note("max|gpu - oracle| / max|u| =", err)
    assert err <= TOL
    # the engine's norm of the start: r0 of the stopping rule
    assert rep["res0"] == pytest.approx(oracle.l2(ss0, n), rel=TOL)
    # the engine's norm after the cycle, against the oracle's residual of
    # the same field
    _, ss1 = oracle.residual(ug, fh, out=False)
    assert rep["res"] == pytest.approx(oracle.l2(ss1, n), rel=TOL)
    del ug
