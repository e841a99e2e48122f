"""Host-side checks of the C ABI that need no GPU: the library loads, every
symbol declared in include/ma.h and include/ma2d.h is exported, and the pure host entry points
(defaults, level hierarchy, footprint, argument validation) behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("ma.h", "ma2d.h"):
        with open(os.path.join(ROOT, "include", h)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(ma2?d?_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_abi():
    names = _declared()
    for n in ("ma_create", "ma_solve", "ma_residual", "ma_vcycle", "ma_destroy",
              "ma_footprint_bytes", "ma_solve_batch", "ma_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1411_7018_amd import _lib
    L = _lib.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert missing == []
    assert set(_lib.EXPORTS) == set(_declared())


def test_defaults_and_levels():
    from paper_1411_7018_amd import _lib as L
    p = L.ma_params_default(128)
    assert (p.n, p.nu1, p.nu2, p.nu0) == (128, 2, 2, 1)
    assert p.order == L.MA_COLOR4 and p.restriction == L.MA_RESTRICT_FULL
    assert p.tol == 1e-8
    assert L.ma_levels(16) == [16, 8, 4, 2]
    assert L.ma_levels(384) == [384, 192, 96, 48, 24, 12, 6, 3]
    assert L.ma_levels(7) == [7]


def test_levels_match_oracle():
    import oracle
    from paper_1411_7018_amd import _lib as L
    for n in (2, 3, 4, 6, 16, 33, 96, 100, 128, 384):
        assert L.ma_levels(n) == oracle.levels(n)


def test_footprint_grows_with_n_and_rejects_invalid():
    from paper_1411_7018_amd import _lib as L
    a = L.ma_footprint_bytes(L.ma_params_default(64))
    b = L.ma_footprint_bytes(L.ma_params_default(128))
    assert 0 < a < b
    # the hierarchy holds the fine residual, the Poisson RHS, the sweep
    # target and the colour-ordered RHS (about 4 fine arrays) plus 5 arrays
    # per coarse level
    n = 128
    fine = (n + 1) ** 3 * 8
    fs = 4 * (((n + 1) // 2 + 63) // 64) * (n - 1) * (n // 2) * 64 * 8
    coarse = 5 * 8 * sum((m + 1) ** 3 for m in L.ma_levels(n)[1:])
    assert 3 * fine + fs <= b <= 3 * fine + fs + coarse + 2**22
    # the mixed form keeps no colour-ordered RHS
    pm = L.ma_params_default(128)
    pm.precision = L.MA_MIXED
    assert L.ma_footprint_bytes(pm) > 0
    bad = L.ma_params_default(1)
    assert L.ma_footprint_bytes(bad) == 0


def test_create_rejects_invalid_params_without_gpu():
    from paper_1411_7018_amd import _lib as L
    for field, val in (("n", 1), ("nu0", 0), ("order", 7), ("precision", 9),
                       ("restriction", 5), ("inner_cycles", 0), ("smoother", 3),
                       ("tile_config", 13), ("tile_config", -1), ("block_n", -2),
                       ("coarse_n", 33), ("max_blocks", 12), ("strip_rows", 5000),
                       ("zsweep_n", -2), ("zsweep_n", 4096), ("fuse_prolong", 1),
                       ("fuse_prolong", -2)):
        p = L.ma_params_default(16)
        setattr(p, field, val)
        with pytest.raises(L.MAError) as ei:
            L.ma_create(p, None)
        assert ei.value.status == L.MA_ERR_ARG
    assert "n must be" in L.ma_last_error(None) or L.ma_last_error(None)


def test_launch_shape_defaults():
    """The knobs that change only the launch structure default to automatic
    (block sweeps on levels up to n = 64, coarse levels up to 16 in one
    kernel), and block_n accepts -1 (never) .. 2048."""
    from paper_1411_7018_amd import _lib as L
    p = L.ma_params_default(128)
    assert (p.smoother, p.tile_config, p.block_n) == (L.MA_SMOOTHER_AUTO, 0, 0)
    assert (p.coarse_n, p.max_blocks, p.strip_rows) == (16, 0, 0)
    for bn in (-1, 0, 32, 2048):
        p.block_n = bn
        assert L.ma_footprint_bytes(p) > 0
    for tc in range(0, 8):
        p.block_n, p.tile_config = 0, tc
        assert L.ma_footprint_bytes(p) > 0
    p.block_n = 2049
    assert L.ma_footprint_bytes(p) == 0


def test_null_handles_are_rejected():
    from paper_1411_7018_amd import _lib as L
    lib = L.lib()
    assert lib.ma_solve(None, None, None, 0.0, 0, None) == L.MA_ERR_ARG
    assert lib.ma_vcycle(None, None, None) == L.MA_ERR_ARG
    assert lib.ma_batch_tick(None, None) == L.MA_ERR_ARG
    assert lib.ma_solve_batch(None, None, None, -1, 0.0, 0, None) == L.MA_ERR_ARG
    lib.ma_destroy(None)
    out = ctypes.c_void_p()
    assert lib.ma_batch_create(0, None, ctypes.byref(out)) == L.MA_ERR_ARG


def test_2d_params_and_footprint():
    from paper_1411_7018_amd import _lib as L
    p = L.ma2d_params_default(256)
    assert (p.n, p.nu1, p.nu2, p.nu0) == (256, 2, 2, 1)
    assert p.order == L.MA2D_RED_BLACK and p.restriction == L.MA_RESTRICT_HALF
    assert p.tol == 1e-6
    fp = L.ma2d_footprint_bytes(p)
    assert 257 ** 2 * 8 * 2 < fp < 257 ** 2 * 8 * 4
    p.order = 7
    assert L.ma2d_footprint_bytes(p) == 0
    with pytest.raises(L.MAError):
        L.ma2d_create(p, None)


def test_stopping_threshold_matches_the_host_test():
    """The device stops a solve when its sum of squares x satisfies x <= T
    (T from sum_threshold); the host stops it when sqrt(x h h h) <= c.  The
    two tests must agree on every double: T passes, the next double up
    fails, and x well below or above T decides the same way on both sides.
    (Host function of the library, reached through its C++ symbol.)"""
    import math

    import numpy as np

    from paper_1411_7018_amd import _lib

    f = getattr(_lib.lib(), "_ZN5mafas13sum_thresholdEdi")
    f.argtypes = [ctypes.c_double, ctypes.c_int]
    f.restype = ctypes.c_double

    def host(x, c, n):
        h = 1.0 / float(n)
        return math.sqrt(x * h * h * h) <= c

    rng = np.random.default_rng(3)
    cases = [(0.0, 2), (1e-300, 16), (3.7e-9, 128), (1.0, 3), (2.5e150, 384)]
    cases += [(float(10.0 ** rng.uniform(-30, 10)), int(rng.integers(2, 1500))) for _ in range(300)]
    for c, n in cases:
        t = f(c, n)
        assert t >= 0.0 and host(t, c, n), (c, n, t)
        up = float(np.nextafter(t, np.inf)) if t < np.finfo(float).max else float("inf")
        assert not host(up, c, n), (c, n, t)
        for x in (t * 0.5, t * 0.999999, up * 1.000001, t * 2.0, 0.0):
            assert host(x, c, n) == (x <= t), (c, n, x, t)
    assert f(-1.0, 16) < 0.0 and f(float("nan"), 16) < 0.0
