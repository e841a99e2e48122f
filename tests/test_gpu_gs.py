"""The standalone nonlinear Gauss-Seidel solver (Section 4's comparison
baseline) on the GPU: same sweep count and result as the oracle's sweeps in
the same colour order, from the Section 4 start 1.01 u."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_gs(p, order, tol=1e-6):
    u = P.initial_guess(p, 1.01 * p.u_exact)
    r0 = math.sqrt(oracle.residual(u, p.f, out=False)[1])
    it = 0
    while True:
        oracle.sweep(u, p.f, order)
        it += 1
        r = math.sqrt(oracle.residual(u, p.f, out=False)[1])
        if r <= tol * r0:
            return u, it


@pytest.mark.parametrize("kind,n,order", [("example4", 8, "4c"), ("example4", 16, "4c"),
                                          ("example5", 12, "8c"), ("example6", 16, "4c")])
def test_gs_solver_matches_oracle(kind, n, order):
    from paper_1411_7018_amd import Solver
    print("[case] gs", kind, n, order, file=sys.stderr, flush=True)
    p = P.make(kind, n)
    want, it = oracle_gs(p, order)
    u = dev(P.initial_guess(p, 1.01 * p.u_exact))
    rep = Solver(n, order=order).gs_solve(u, dev(p.f), tol=1e-6)
    assert rep["converged"] == 1 and rep["cycles"] == it
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_gs_solver_not_converged_reports():
    from paper_1411_7018_amd import Solver, _lib as L
    p = P.example4(16)
    u = dev(P.initial_guess(p, 1.01 * p.u_exact))
    with pytest.raises(L.MAError) as ei:
        Solver(16).gs_solve(u, dev(p.f), tol=1e-6, max_sweeps=5)
    assert ei.value.status == L.MA_ERR_NOT_CONVERGED
    assert ei.value.report["cycles"] == 5 and 0 < ei.value.report["rel_res"] < 1
