"""The allocation-free residual (ma_residual_noalloc) through the C ABI
against ma_residual of a solver: the same residual field bit for bit and the
same norm, on two calls in a row with the second grid smaller than the
first (the static scratch keeps the first call's partials), and sizes
beyond its maximum refused before any GPU work."""
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


def _data(n, seed):
    p = P.exp_cos(n, seed=seed)
    rng = np.random.default_rng(seed)
    u = P.initial_guess(p, p.u_exact * (1.0 + 1e-3 * rng.standard_normal(p.u_exact.shape)))
    return torch.from_numpy(u).cuda(), torch.from_numpy(p.f).cuda()


def _noalloc(n, u, f, with_r=True):
    from paper_1411_7018_amd import _lib as L
    r = torch.full_like(u, np.nan) if with_r else None
    l2 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    L.ma_residual_noalloc(n, u.data_ptr(), f.data_ptr(), r.data_ptr() if with_r else None,
                          l2.data_ptr(), stream)
    torch.cuda.synchronize()
    return r, float(l2.item())


def test_noalloc_matches_ma_residual_two_calls_second_smaller():
    from paper_1411_7018_amd import Solver
    for n, seed in ((96, 1), (40, 2)):
        note("noalloc residual", n)
        u, f = _data(n, seed)
        r_ref = torch.empty_like(u)
        l2_ref = Solver(n).residual(u, f, r_ref)
        r, l2 = _noalloc(n, u, f)
        assert torch.equal(r, r_ref)
        assert l2 == pytest.approx(l2_ref, rel=1e-15, abs=0.0)
        # without the field, the norm alone
        _, l2b = _noalloc(n, u, f, with_r=False)
        assert l2b == l2


def test_noalloc_allocates_nothing_after_first_use():
    """Once the library is loaded on the device, calls take no device memory:
    the free memory the runtime reports is the same before and after."""
    from paper_1411_7018_amd import _lib as L
    n = 64
    u, f = _data(n, 3)
    _noalloc(n, u, f)
    r = torch.empty_like(u)
    l2 = torch.empty(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    for _ in range(5):
        L.ma_residual_noalloc(n, u.data_ptr(), f.data_ptr(), r.data_ptr(), l2.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    assert free2 == free1


@pytest.mark.parametrize("n", [1, 513, 1024])
def test_noalloc_rejects_sizes_beyond_its_scratch(n):
    from paper_1411_7018_amd import _lib as L
    u = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(L.MAError) as ei:
        L.ma_residual_noalloc(n, u.data_ptr(), u.data_ptr(), None, u.data_ptr(), None)
    assert ei.value.status == L.MA_ERR_ARG
    assert "2..512" in L.ma_last_error(None)
