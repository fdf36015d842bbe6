"""The allocation-free periodic search (fixed device scratch) against the
workspace form of the same search, through the C ABI: identical records on
two calls in a row, the second over a smaller input (fewer periods and a
shorter curve), so stale scratch contents from the first call cannot leak
into the second."""

import numpy as np
import pytest

from synthlc import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_20875_amd as cm
    cm._abi.load()
    return cm


def _prepare(cm, wl):
    import torch
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    model = cm.template_resample(wl.dense, wl.n_model)
    flux, ivar, _ = cm.resample(grid, wl.t, wl.f, wl.sigma)
    fold = cm.linear_search(grid, flux, ivar, model)
    torch.cuda.synchronize()
    return grid, fold


def _host(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _same(a, b):
    for k in ("lr", "epoch", "dur", "depth", "depth_var"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_noalloc_equals_workspace_form_twice(cm):
    import torch
    big = W.tiny_single()
    small = W.small_random(5, n_obs=3000, n_dur=4, n_per=300, p_range=(0.6, 3.0), dur_h=(1.0, 3.0))
    lim = None
    for name, wl in (("tiny_single", big), ("small_random", small)):
        print(f"[noalloc] {name}: K={len(wl.periods)}", flush=True)
        grid, fold = _prepare(cm, wl)
        lim = cm.periodic_search_noalloc_limit(grid)
        assert lim >= len(wl.periods)
        ref = _host(cm.periodic_search(grid, fold, wl.periods))
        got = cm.periodic_search_noalloc(grid, fold, wl.periods)
        torch.cuda.synchronize()
        got = _host(got)
        _same(got, ref)
        assert (got["epoch"] >= 0).sum() > 0
        # a subset of the periods: the others get the null record
        sub = np.arange(0, len(wl.periods), 3, dtype=np.int64)
        ref_s = _host(cm.periodic_search(grid, fold, wl.periods, subset=sub))
        got_s = _host(cm.periodic_search_noalloc(grid, fold, wl.periods, subset=sub))
        torch.cuda.synchronize()
        _same(got_s, ref_s)


def test_noalloc_rejects_more_periods_than_the_scratch_holds(cm):
    import torch
    wl = W.small_random(6, n_obs=1500, n_dur=2, n_per=64, p_range=(0.6, 2.0), dur_h=(1.0, 2.0))
    grid, fold = _prepare(cm, wl)
    lim = cm.periodic_search_noalloc_limit(grid)
    periods = torch.full((lim + 1,), 1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(cm.CetraError, match="scratch"):
        cm.periodic_search_noalloc(grid, fold, periods)
