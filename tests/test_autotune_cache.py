"""The autotuner's cache, on the host: an entry for the shape class and
architecture is applied without any device work; an entry with an invalid
tuning is ignored; a class with no entry needs the caller's data (argument
check before any device call)."""

import ctypes
import json
import os

import pytest


@pytest.fixture(scope="module")
def lib():
    from paper_2503_20875_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2503_20875_amd import build
        build.build()
    return _abi.load()


def test_cache_hit_applies_the_entry_without_a_device(lib, tmp_path):
    import paper_2503_20875_amd as cm
    from paper_2503_20875_amd import _abi
    from paper_2503_20875_amd.autotune import shape_class
    grid = cm.grid_plan(0.0, 90.0, 20.0 / 86400, [0.05, 0.1, 0.2])
    sc = shape_class(grid, 50_000, arch="gfx950")
    assert sc.log2_t0 == (grid.n_t0 - 1).bit_length() and sc.log2_periods == 16 and sc.n_dur == 3
    entry = dict(arch="gfx950", log2_t0=sc.log2_t0, n_dur=3, log2_periods=16, fold_period_block=4,
                 fold_wgs_per_cu=2, fold_units_per_wg=8, fold_variant=0, linear_windows=2, fold_ms=1.5,
                 linear_ms=0.25)
    bad = dict(entry, log2_periods=15, fold_period_block=5)  # invalid tuning: ignored
    other = dict(entry, arch="gfx942", fold_period_block=16)
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"format": "cetra-autotune-1", "entries": [other, bad, entry]}, indent=1))
    out, fms, lms, hit = _abi.Tuning(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    try:
        rc = lib.cetra_autotune(None, ctypes.byref(sc), ctypes.byref(grid), None, None, None, None, None, 50_000,
                                None, 0, str(path).encode(), ctypes.byref(out), ctypes.byref(fms),
                                ctypes.byref(lms), ctypes.byref(hit))
        assert rc == 0, lib.cetra_last_error()
        assert hit.value == 1 and fms.value == 1.5 and lms.value == 0.25
        got = {k: getattr(out, k) for k in ("fold_period_block", "fold_wgs_per_cu", "fold_units_per_wg",
                                            "fold_variant", "linear_windows")}
        assert got == {k: entry[k] for k in got}
        assert cm.get_tuning() == got
        # the class with the invalid entry: a miss, which needs the caller's data
        sc2 = shape_class(grid, 20_000, arch="gfx950")
        assert sc2.log2_periods == 15
        rc = lib.cetra_autotune(None, ctypes.byref(sc2), ctypes.byref(grid), None, None, None, None, None, 20_000,
                                None, 0, str(path).encode(), ctypes.byref(out), None, None, ctypes.byref(hit))
        assert rc == -1 and b"NULL" in lib.cetra_last_error()
        assert cm.get_tuning() == got  # unchanged
    finally:
        cm.reset_tuning()
