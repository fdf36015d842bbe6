"""The library's host-side grid calls (cetra_period_grid,
cetra_duration_limits, cetra_keplerian_jrange) against the grid oracle.
They are pure FP64 host code, so they run without a GPU.  Periods and
limits agree to a few units of FP64 rounding; duration-index ranges agree
exactly except where a duration sits on a limit to within that rounding."""

import numpy as np
import pytest

from oracle import grids as og
from synthlc import workloads as W


@pytest.fixture(scope="module")
def cm():
    import paper_2503_20875_amd as cm
    cm._abi.load()
    return cm


@pytest.mark.parametrize("span,p_min,p_max,rho,os_", [(90.0, 0.5, 45.0, 1.41, 3.0), (730.5, 1.0, 400.0, 1.41, 2.0),
                                                      (27.4, 0.3, 13.7, 5.0, 5.0)])
def test_period_grid_matches_oracle(cm, span, p_min, p_max, rho, os_):
    got = cm.period_grid(span, p_min, p_max, rho, os_)
    want = og.period_grid(span, p_min, p_max, rho, os_)
    assert got.shape == want.shape
    assert np.max(np.abs(got / want - 1.0)) < 1e-13


def test_period_grid_rejects_bad_ranges(cm):
    for args in ((90.0, 45.0, 0.5, 1.41, 3.0), (0.0, 0.5, 45.0, 1.41, 3.0), (90.0, 0.5, 45.0, -1.0, 3.0),
                 (90.0, 0.5, 45.0, 1.41, 0.0)):
        with pytest.raises(cm.CetraError):
            cm.period_grid(*args)


def test_duration_limits_match_oracle(cm):
    for P in (0.02, 0.5, 3.0, 30.0, 365.25):
        for rho_min, rho_max, k, b in ((0.5, 3.0, 0.2, 0.9), (1.41, 1.41, 0.0092, 0.0), (0.05, 60.0, 0.3, 0.99)):
            lo, hi = cm.duration_limits(P, rho_min, rho_max, k, b)
            olo, ohi = og.duration_limits(P, rho_min, rho_max, k, b)
            assert lo == pytest.approx(olo, rel=1e-13, abs=1e-300) and hi == pytest.approx(ohi, rel=1e-13)
    with pytest.raises(cm.CetraError):
        cm.duration_limits(3.0, 3.0, 0.5)  # rho_min > rho_max


def test_keplerian_jrange_matches_oracle(cm):
    wl = W.high_cadence()
    sel = np.arange(0, len(wl.periods), 7)
    periods = wl.periods[sel]
    got = cm.keplerian_jrange(periods, wl.durations, 0.5, 3.0, 0.2, 0.9)
    want = og.keplerian_jrange(periods, wl.durations, 0.5, 3.0, 0.2, 0.9)
    bad = np.flatnonzero(np.any(got != want, axis=1))
    for k in bad:  # only a duration lying on a limit may be decided differently
        lo, hi = og.duration_limits(periods[k], 0.5, 3.0, 0.2, 0.9)
        assert np.min(np.abs(np.log(wl.durations / np.array([[lo], [hi]])))) < 1e-12
    assert bad.size <= 2
    # every period keeps at least one duration on this grid, and some lose some
    assert np.all(got[:, 0] <= got[:, 1])
    assert np.any(got[:, 0] > 0) and np.any(got[:, 1] < len(wl.durations) - 1)


@pytest.mark.parametrize("name", ["tiny", "high_cadence", "long_baseline"])
@pytest.mark.parametrize("fraction", [0.01, 0.03])
def test_epoch_strides_match_oracle(cm, name, fraction):
    """The host's duration-scaled epoch strides equal the grid oracle's
    exactly on each workload's grid."""
    if name == "long_baseline":
        sh = W.long_baseline_shape()
        g = cm.grid_plan(0.0, sh["span"], sh["cadence"], sh["durations"], 0.0, 1024)
        durs = sh["durations"]
    else:
        wl = W.WORKLOADS[name]()
        g = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, 1024)
        durs = wl.durations
    got = cm.epoch_strides(g, fraction)
    want = og.epoch_strides(durs, g.t0_step, fraction)
    assert np.array_equal(got, want)
    assert got[0] == max(1, int(fraction / 0.01 + 1e-9))


def test_epoch_strides_reject_bad_fractions(cm):
    wl = W.tiny_single()
    g = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, 1024)
    for bad in (0.0, -0.01, float("nan"), float("inf")):
        with pytest.raises(cm.CetraError, match="fraction"):
            cm.epoch_strides(g, bad)
