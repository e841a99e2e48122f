"""FMG-FAS (Algorithm 2) on the GPU against the oracle: the FMG iteration
alone, full solves under the Section 4 protocol (r^0 of the zero-interior
start, the FMG iteration as the first cycle), Table 3's 'Iter' = 1, and the
batched / resident / mixed-precision paths."""
import sys

import numpy as np
import pytest

import oracle
from paper_1411_7018_amd import problems as P

pytestmark = pytest.mark.gpu
TOL = 1e-12          # FP64 parity bar (relative max-norm), as for the V-cycle
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def note(*args):
    print("[case]", *args, file=sys.stderr, flush=True)


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n,kind,order", [(2, "example4", "4c"), (3, "exp_cos", "4c"),
                                          (4, "quadratic", "4c"), (6, "exp_cos", "4c"),
                                          (8, "example4", "4c"), (12, "exp_cos", "8c"),
                                          (16, "example4", "4c"), (24, "exp_cos", "4c"),
                                          (33, "quadratic", "4c"), (40, "exp_cos", "4c"),
                                          (64, "exp_cos", "4c")])
def test_fmg_matches_oracle(n, kind, order):
    from paper_1411_7018_amd import Solver
    note("fmg", n, kind, order)
    p = P.make(kind, n, 17)
    u0 = P.initial_guess(p, 0.7)          # the interior is not read
    want = u0.copy()
    nc_o = oracle.fmg(want, p.f, oracle.params(order=order))
    u = dev(u0)
    nc_g = Solver(n, order=order).fmg(u, dev(p.f))
    assert relmax(host(u), want) <= TOL
    assert nc_g == nc_o


@pytest.mark.parametrize("n,kind", [(8, "example4"), (16, "exp_cos"), (24, "quadratic"),
                                    (48, "exp_cos")])
def test_solve_with_fmg_start_matches_oracle(n, kind):
    from paper_1411_7018_amd import Solver
    note("fmg solve", n, kind)
    p = P.make(kind, n, 5)
    want = P.initial_guess(p)
    st, rep_o, _ = oracle.solve(want, p.f, oracle.params(init="fmg", tol=1e-9))
    assert st == 0
    u = dev(P.initial_guess(p, 0.25))
    rep = Solver(n).solve(u, dev(p.f), tol=1e-9, init="fmg")
    assert rep["converged"] == 1 and rep["cycles"] == rep_o.cycles
    assert rep["res0"] == pytest.approx(rep_o.res0, rel=1e-12)
    assert relmax(host(u), want) <= TOL


@pytest.mark.parametrize("N", [8, 16, 32])
def test_table3_one_fmg_iteration_gpu(N):
    """Example 4 at the Section 4 tolerance 1e-6: one FMG-FAS iteration
    suffices ('Iter' = 1 in Table 3), here with the 4-colour ordering."""
    from paper_1411_7018_amd import Solver
    note("table3 fmg", N)
    p = P.example4(N)
    u = dev(P.initial_guess(p))
    rep = Solver(N).solve(u, dev(p.f), tol=1e-6, init="fmg")
    assert rep["converged"] == 1 and rep["cycles"] == 1
    assert rep["rel_res"] <= 1e-6
    err = np.abs(host(u) - p.u_exact).max()
    e_lim = {8: 1.157e-3, 16: 2.977e-4, 32: 7.55e-5}[N]   # converged discrete error
    assert err <= 2.0 * e_lim


def test_fmg_batch_and_resident_equal_solo():
    from paper_1411_7018_amd import Solver
    from paper_1411_7018_amd.batch import ResidentBatch, solve_batch
    note("fmg batch")
    specs = [("exp_cos", 16, 1), ("quadratic", 24, 2), ("example4", 32, 3), ("exp_cos", 12, 4)]
    probs = [P.make(k, n, s) for k, n, s in specs]
    want = []
    for p in probs:
        u = dev(P.initial_guess(p))
        Solver(p.n).solve(u, dev(p.f), tol=1e-9, init="fmg")
        want.append(host(u))
    us = [dev(P.initial_guess(p)) for p in probs]
    st, reps = solve_batch([Solver(p.n) for p in probs], us, [dev(p.f) for p in probs],
                           tol=1e-9, init="fmg")
    assert st == 0
    for u, w in zip(us, want):
        assert np.array_equal(host(u), w)
    b = ResidentBatch(4)
    live = {}
    for p in probs:
        sv = Solver(p.n)
        u = dev(P.initial_guess(p))
        live[b.add(sv, u, dev(p.f), tol=1e-9, init="fmg")] = (sv, u)
    done = {}
    for _ in range(100):
        done.update(b.tick())
        if len(done) == len(probs):
            break
    assert all(c == 1 for c in done.values()) and len(done) == len(probs)
    for slot, (sv, u) in live.items():
        assert np.array_equal(host(u), want[slot])


def test_mixed_with_fmg_start_reaches_oracle_limit():
    """Mixed precision from the FMG start, run to its round-off floor (the
    Section 4 r^0 is the residual of the zero-interior start, so a relative
    tolerance stops far earlier): agrees with the FP64 oracle limit."""
    from paper_1411_7018_amd import Solver, _lib as L
    note("fmg mixed")
    n = 32
    p = P.exp_cos(n, seed=21)
    lim = P.initial_guess(p)
    oracle.solve_limit(lim, p.f)
    u = dev(P.initial_guess(p))
    s = Solver(n, precision="mixed", max_cycles=24)
    with pytest.raises(L.MAError) as ei:          # an unreachable tolerance
        s.solve(u, dev(p.f), tol=1e-30, init="fmg")
    assert ei.value.status == L.MA_ERR_NOT_CONVERGED
    assert np.abs(host(u) - lim).max() <= 1e-10


def test_fmg_flags_exclude_each_other():
    from paper_1411_7018_amd import Solver, _lib as L
    p = P.example4(8)
    s = Solver(8)
    with pytest.raises(L.MAError):
        L.ma_solve(s.handle, s._grid(dev(P.initial_guess(p))), s._grid(dev(p.f)), -1.0,
                   L.MA_INIT_POISSON | L.MA_INIT_FMG)
