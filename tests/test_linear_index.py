"""The linear search's template lookup replaces the clamp of the
nearest-sample index to M - 1 by copies of the last sample at indices M ..
M + 3 (the device table).  That is exact only if the unclamped 32.32 index of
a point inside its window never exceeds M + 3; this checks, with exact
integer arithmetic on the window rule (Sec. 2.1.2, Sec. 2.2), that it never
exceeds M on every window of the benchmark and test workloads."""

import numpy as np
import pytest

from synthlc import workloads as W

TWO32 = 2 ** 32


def max_index(g):
    """Largest unclamped index (phase + (L - 1) G) >> 32 over all non-null
    windows, with the window bounds and phase computed as the grid plan
    defines them (FP64, round half away from zero for the phase)."""
    c, dt, M = g.cadence, g.t0_step, g.n_model
    t_end = (g.n - 1) * c
    i = np.arange(g.n_t0, dtype=np.float64)
    worst = 0
    for j in range(g.n_dur):
        D = g.durations[j]
        ts = i * dt - 0.5 * D
        te = ts + D
        ok = ~((ts < 0.0) | (te > t_end))
        lo = np.ceil(ts[ok] / c)
        hi = np.floor(te[ok] / c)
        keep = lo <= hi
        lo, hi, tsk = lo[keep], hi[keep], ts[ok][keep]
        x = TWO32 * (((lo * c - tsk) / D) * M)
        phase = np.maximum(np.floor(x + 0.5), 0.0).astype(np.uint64)  # llround of a non-negative value
        G = np.uint64(int(g.dur_step_fx[j]))
        L = (hi - lo).astype(np.uint64)
        k_last = (phase + L * G) >> np.uint64(32)
        worst = max(worst, int(k_last.max()) if k_last.size else 0)
    return worst


@pytest.mark.parametrize("name", ["tiny", "high_cadence", "small"])
def test_template_index_never_exceeds_m(name):
    import oracle
    wl = {"tiny": W.tiny_single, "high_cadence": W.high_cadence,
          "small": lambda: W.small_random(3, n_obs=4000, n_dur=6, n_per=10)}[name]()
    g = oracle.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model)
    k = max_index(g)
    assert k <= g.n_model, (name, k)


def test_template_index_bound_on_the_survey_and_long_grids():
    import oracle
    from paper_2503_20875_amd import _abi  # noqa: F401  (grid shapes only)
    sh = W.long_baseline_shape()
    g = oracle.grid_plan(0.0, sh["span"], sh["cadence"], sh["durations"], 1024)
    assert max_index(g) <= 1024
    for c in W.survey_subset(6, n_min=5000, n_max=120000):
        g = oracle.grid_plan(c.t[0], c.t[-1], c.cadence, c.durations, c.n_model)
        assert max_index(g) <= c.n_model
