"""The z-stream sweep (all four colour phases of a sweep in one launch, each
workgroup walking a column of the grid plane by plane with the phases two
planes apart, out of place) at the sizes it is built for: bitwise equal to
the colour-phase kernels over pairs of sweeps at 129^3, 257^3 and 385^3.
The colour-phase form is itself checked node by node against the oracle at
these sizes (test_gpu_fullsize), and the engine's V-cycle with z-stream
sweeps on its finest level against the oracle's V-cycle (test_gpu_benchshape)."""
import sys

import numpy as np
import pytest

from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ZS_CONFIGS = (8, 9, 10, 11)


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def solver(n, **kw):
    from paper_1411_7018_amd import Solver
    return Solver(n, **kw)


@pytest.mark.parametrize("n", [128, 256, 384])
def test_zsweep_full_size_bitwise_vs_colour(n):
    note("z-stream sweep full size", n)
    u0, f, ue = P.make_device("exp_cos", n, 7000 + n, exact=True)
    # a smooth convex start: the solution plus a bump that vanishes on the boundary
    t = torch.arange(n + 1, dtype=torch.float64, device="cuda") / n
    s = torch.sin(np.pi * t)
    start = ue + 0.01 * s[:, None, None] * s[None, :, None] * s[None, None, :]
    del ue
    uc = start.clone()
    solver(n, smoother="color").sweep(uc, f, 2)
    for cfg in ZS_CONFIGS:
        uz = start.clone()
        solver(n, smoother="fused", tile_config=cfg).sweep(uz, f, 2)
        torch.cuda.synchronize()
        assert torch.equal(uz, uc), cfg
        del uz
