"""Host-side pieces of the period-recovery experiment (Sec. 4.1, Table 1):
its light-curve layout, noise level, injections, recovery criterion and
search grids, checked against the paper's statement of the test and against
the grid oracle (no GPU)."""

import numpy as np
import pytest

from oracle import grids as og
from paper_2503_20875_amd import recovery as R
from synthlc import workloads as W


def test_times_span_cadence_and_gap():
    """173 d at 600 s, nothing inside the 7-d gap from day 90."""
    t = R.times()
    c = 600.0 / 86400.0
    assert t[0] == 0.0 and t[-1] == pytest.approx(173.0)
    assert not np.any((t >= 90.0) & (t < 97.0))
    d = np.diff(t)
    assert np.allclose(d[d < 1.0], c) and np.count_nonzero(d > 1.0) == 1
    assert t.size == round(173.0 / c) + 1 - round(7.0 / c)


def test_noise_level_is_per_hour():
    """Reading T1: white noise whose one-hour mean (six 600-s points) has the
    stated standard deviation."""
    rng = np.random.default_rng(0)
    for level in R.NOISE_LEVELS:
        x = rng.normal(0.0, R.noise_sigma(level), 6 * 200_000)
        hourly = x.reshape(-1, 6).mean(axis=1)
        assert hourly.std() == pytest.approx(level * 1e-6, rel=0.01)


def test_recovery_criterion():
    """Within 1% of P, P/2 or 2P (Sec. 4.1), nothing else."""
    P = 10.0
    for ok in (10.0, 10.09, 9.91, 5.04, 4.96, 20.19, 19.81):
        assert R.recovered(ok, P), ok
    for bad in (10.11, 9.89, 5.06, 4.94, 20.21, 19.79, 3.333, 30.0, float("nan")):
        assert not R.recovered(bad, P), bad


def test_injections_follow_the_recipe():
    """Periods uniform over 1-86.5 d, epochs within one period, durations
    between the Keplerian limits of the grid oracle (density 0.5-3 g/cm^3,
    k <= 0.2, b <= 0.9), depths log-uniform over 50-1000 ppm."""
    lim = lambda P: og.duration_limits(P, R.RHO[0], R.RHO[1], R.K_MAX, R.B_MAX)
    inj = R.draw(np.random.default_rng(1), lim, 4000)
    P, e, d, dep = inj.T
    assert P.min() >= 1.0 and P.max() <= 86.5
    assert abs(np.mean(P) - 43.75) < 1.5
    assert np.all((e >= 0) & (e < P))
    for k in range(0, 4000, 97):
        lo, hi = lim(P[k])
        assert lo <= d[k] <= hi
    assert dep.min() >= 50e-6 and dep.max() <= 1000e-6
    assert abs(np.mean(np.log(dep)) - 0.5 * (np.log(50e-6) + np.log(1000e-6))) < 0.05


def test_injected_depth_is_the_maximum_offset():
    """The stated depth is the largest flux offset of the injected shape."""
    t = np.linspace(9.5, 10.5, 200001)
    sig = W.inject(t, W.Injection(period=37.0, epoch=10.0, duration=0.25, depth=4e-4))
    assert sig.max() == pytest.approx(4e-4, rel=1e-5)
    assert sig[np.abs(t - 10.0) > 0.126].max() == 0.0


def test_search_grids_match_the_grid_oracle():
    """The library's default grids for this span equal the grid oracle's:
    24 log-spaced durations 0.6-30 h, the optimal period grid over 1-86.5 d
    at solar density and oversampling 3, and the per-period Keplerian
    duration ranges."""
    import paper_2503_20875_amd as cm
    t = R.times()
    durs, periods, jr = R.search_grids(cm, t)
    assert len(durs) == 24 and durs[0] == pytest.approx(0.025) and durs[-1] == pytest.approx(1.25)
    ref = og.period_grid(t[-1] - t[0], 1.0, 86.5, cm.SOLAR_DENSITY, 3.0)
    assert len(periods) == len(ref) and np.allclose(periods, ref, rtol=1e-12)
    assert np.array_equal(jr, og.keplerian_jrange(periods, durs, R.RHO[0], R.RHO[1], R.K_MAX, R.B_MAX))


def test_light_curve_is_offset_plus_noise():
    """The search input is 1 - (1 - signal + noise) as FP32 offsets, with the
    per-point sigma of the level."""
    rng = np.random.default_rng(4)
    sig = np.zeros(1000)
    sig[100:110] = 5e-4
    f, s = R.light_curve(sig, 160.0, rng)
    assert f.dtype == np.float32 and s.dtype == np.float32
    assert np.all(s == np.float32(R.noise_sigma(160.0)))
    noise = np.random.default_rng(4).normal(0.0, R.noise_sigma(160.0), 1000)
    assert np.allclose(f, (sig - noise).astype(np.float32), atol=1e-9)
