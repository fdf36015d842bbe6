"""The library's autotuner times its candidates on the caller's data,
applies and caches the fastest; a second call takes it from the cache; the
search under the tuning returns the records of the default tuning."""

import json

import numpy as np
import pytest

from synthlc import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_measures_caches_and_keeps_results(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_20875_amd as cm
    from paper_2503_20875_amd.autotune import tune
    wl = W.tiny_single()
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    model = cm.template_resample(torch.as_tensor(wl.dense, device="cuda"), wl.n_model)
    flux, ivar, _ = cm.resample(grid, wl.t, wl.f, wl.sigma)
    fold = cm.linear_search(grid, flux, ivar, model)
    per = torch.as_tensor(wl.periods, device="cuda")
    cm.reset_tuning()
    ref = {k: v.cpu().numpy() for k, v in cm.periodic_search(grid, fold, per).items()}
    ref_fold = fold.cpu().numpy()
    cache = tmp_path / "autotune.json"
    print("[autotune] tiny workload, timing", flush=True)
    try:
        r1 = tune(grid, flux, ivar, model, fold, per, cache_path=cache)
        assert not r1["from_cache"] and r1["fold_ms"] > 0 and r1["linear_ms"] > 0
        assert cm.get_tuning() == r1["tuning"]
        entries = json.loads(cache.read_text())["entries"]
        assert len(entries) == 1 and entries[0]["arch"].startswith("gfx")
        assert np.array_equal(fold.cpu().numpy(), ref_fold)  # re-computed, same values
        got = {k: v.cpu().numpy() for k, v in cm.periodic_search(grid, fold, per).items()}
        for k in ref:
            assert np.array_equal(got[k], ref[k], equal_nan=True), k
        cm.reset_tuning()
        print("[autotune] from the cache", flush=True)
        r2 = tune(grid, flux, ivar, model, fold, per, cache_path=cache)
        assert r2["from_cache"] and r2["tuning"] == r1["tuning"] and cm.get_tuning() == r1["tuning"]
    finally:
        cm.reset_tuning()
