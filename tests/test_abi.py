"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, validates arguments before enqueueing anything, and its
host-only grid plan agrees with the oracle's (separately written) one."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cetra.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cetra_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2503_20875_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2503_20875_amd import build
        build.build()
    return _abi.load()


def test_exports_every_declared_symbol(lib):
    from paper_2503_20875_amd import _abi
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), f"{n} declared in cetra.h but not exported"
    assert set(names) == set(_abi.SIGNATURES), "binding and header disagree on the export list"


def test_version_and_status_strings(lib):
    assert lib.cetra_version() == 100
    assert lib.cetra_status_string(0) == b"ok"
    assert lib.cetra_status_string(-3) == b"workspace too small"


def test_grid_plan_matches_oracle(lib, ora):
    import paper_2503_20875_amd as cm
    from synthlc import workloads as W
    for wl in (W.tiny_single(), W.small_random(3)):
        g = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
        o = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model)
        for f in ("t_first", "cadence", "t_origin", "t0_step", "n_pad", "n_data", "n", "n_t0", "n_dur", "n_model"):
            assert getattr(g, f) == getattr(o, f), f
        assert list(g.durations) == list(o.durations)
        assert list(g.dur_step_fx) == list(o.dur_step_fx)


def test_grid_plan_validation(lib):
    import paper_2503_20875_amd as cm
    with pytest.raises(cm.CetraError, match="ascending"):
        cm.grid_plan(0.0, 10.0, 0.01, [0.2, 0.1])
    with pytest.raises(cm.CetraError, match="cadence"):
        cm.grid_plan(0.0, 10.0, 0.0, [0.1])
    with pytest.raises(cm.CetraError, match="n_model"):
        cm.grid_plan(0.0, 10.0, 0.01, [0.1], n_model=5000)
    with pytest.raises(cm.CetraError, match="reference times|2\\^32"):
        cm.grid_plan(0.0, 1e6, 1e-4, [1e-4, 2e-4])


def test_calls_reject_bad_arguments_without_a_gpu(lib):
    """Argument checks run on the host before any launch."""
    from paper_2503_20875_amd import _abi
    g = _abi.Grid()
    rc = lib.cetra_linear_search(None, ctypes.byref(g), None, None, None, None, None, None, None)
    assert rc == -1 and b"not planned" in lib.cetra_last_error() or rc == -1
    import paper_2503_20875_amd as cm
    grid = cm.grid_plan(0.0, 1.0, 0.01, [0.05, 0.1])
    rc = lib.cetra_linear_search(None, ctypes.byref(grid), None, None, None, None, None, None, None)
    assert rc == -1 and b"NULL" in lib.cetra_last_error()
    need = ctypes.c_size_t()
    assert lib.cetra_periodic_workspace(ctypes.byref(grid), 1000, ctypes.byref(need)) == 0
    assert need.value >= 1000 * 8
    rc = lib.cetra_periodic_search(None, ctypes.byref(grid), ctypes.c_void_p(8), ctypes.c_void_p(8), 1000, None,
                                   None, 0, ctypes.c_void_p(8), need.value - 1, ctypes.c_void_p(8),
                                   ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8))
    assert rc == -3


def test_tuning_roundtrip_and_validation(lib):
    import paper_2503_20875_amd as cm
    cm.reset_tuning()
    assert cm.get_tuning() == dict(fold_period_block=8, fold_wgs_per_cu=8, fold_units_per_wg=4, fold_variant=2,
                                   linear_windows=4)
    cm.set_tuning(4, 6, 2, 0, 2)
    assert cm.get_tuning() == dict(fold_period_block=4, fold_wgs_per_cu=6, fold_units_per_wg=2, fold_variant=0,
                                   linear_windows=2)
    with pytest.raises(cm.CetraError, match="linear_windows"):
        cm.set_tuning(4, 6, 2, 0, 3)
    with pytest.raises(cm.CetraError, match="fold_period_block"):
        cm.set_tuning(5, 6, 2)
    with pytest.raises(cm.CetraError, match="fold_variant"):
        cm.set_tuning(4, 6, 2, 1)
    assert cm.get_tuning()["fold_period_block"] == 4  # unchanged after a rejected call
    cm.reset_tuning()
    assert cm.get_tuning()["fold_period_block"] == 8


def test_noalloc_limit_and_range_error_without_a_gpu(lib):
    """The allocation-free periodic search reports its period limit and
    rejects a larger request on the host, before touching the device."""
    import paper_2503_20875_amd as cm
    from paper_2503_20875_amd import _abi
    grid = cm.grid_plan(0.0, 1.0, 0.01, [0.05, 0.1])
    lim = cm.periodic_search_noalloc_limit(grid)
    assert cm.periodic_workspace(grid, lim) <= 16 << 20 < cm.periodic_workspace(grid, lim + 1)
    assert lim >= 400_000  # the two-year, 400 000-period search fits
    rc = lib.cetra_periodic_search_noalloc(None, ctypes.byref(grid), None, None, lim + 1, None, None, 0,
                                           None, None, None, None, None)
    assert rc == -2 and b"scratch" in lib.cetra_last_error()
    rc = lib.cetra_periodic_search_noalloc(None, ctypes.byref(grid), None, None, -1, None, None, 0,
                                           None, None, None, None, None)
    assert rc == -1
    assert _abi.SIGNATURES["cetra_periodic_search_noalloc"][0] is ctypes.c_int


def test_conv_backward_workspace_size(lib):
    """cetra_conv1d_bwd_partial_floats (host only): one slab of 64 k32 + 64
    floats per weight-gradient workgroup, with the most 256-position chunks
    per workgroup (8, 4, 2 or 1) that still give 256 workgroups."""
    def expected(cin, L, B):
        k32 = (9 * cin + 31) // 32 * 32
        cpw = 1
        for c in (8, 4, 2):
            if -(-L // (256 * c)) * B >= 256:
                cpw = c
                break
        return -(-L // (256 * cpw)) * B * (64 * k32 + 64)
    for cin, L, B in ((64, 8192, 32), (16, 8192, 32), (16, 4096, 32), (64, 8192, 256), (64, 300, 2), (16, 1, 1),
                      (64, 8192, 1), (64, 65536, 4)):
        assert lib.cetra_conv1d_bwd_partial_floats(cin, L, B) == expected(cin, L, B), (cin, L, B)
    assert lib.cetra_conv1d_bwd_partial_floats(64, 8192, 32) == 256 * (64 * 576 + 64)
    for bad in ((32, 100, 1), (64, 0, 1), (64, 100, 0)):
        assert lib.cetra_conv1d_bwd_partial_floats(*bad) == -1
