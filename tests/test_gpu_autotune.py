"""The launch-tuning search picks one of its candidates, applies it, and the
search under it returns the records of the default tuning."""

import numpy as np
import pytest

from synthlc import workloads as W

pytestmark = pytest.mark.gpu


def test_tune_fold_applies_a_candidate():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_20875_amd as cm
    from paper_2503_20875_amd.autotune import tune_fold
    wl = W.tiny_single()
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    model = cm.template_resample(torch.as_tensor(wl.dense, device="cuda"), wl.n_model)
    flux, ivar, _ = cm.resample(grid, wl.t, wl.f, wl.sigma)
    fold = cm.linear_search(grid, flux, ivar, model)
    per = torch.as_tensor(wl.periods, device="cuda")
    cm.reset_tuning()
    ref = {k: v.cpu().numpy() for k, v in cm.periodic_search(grid, fold, per).items()}
    cands = [(4, 8, 4, 0), (8, 8, 4, 0), (4, 8, 16, 2), (4, 8, 4, 2)]
    print("[autotune] tiny workload", flush=True)
    try:
        cfg, times = tune_fold(grid, fold, per, candidates=cands, repeats=1)
        assert tuple(cfg.values()) in cands and set(times) == set(cands)
        assert cm.get_tuning() == cfg
        got = {k: v.cpu().numpy() for k, v in cm.periodic_search(grid, fold, per).items()}
        for k in ref:
            assert np.array_equal(got[k], ref[k], equal_nan=True), k
    finally:
        cm.reset_tuning()
