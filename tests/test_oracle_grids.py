"""Pins of the grid oracle (oracle/grids.py) against astronomy and closed
forms, not against itself: Kepler's third law for the Earth's orbit, the
duration of the Earth's transit across the Sun, the small-angle limit of the
duration formula, its degenerate cases, and the optimal-sampling criterion
that defines the period grid."""

import numpy as np
import pytest

from oracle import grids as og

RHO_SUN = 1.41          # g cm^-3 (M_sun / (4/3 pi R_sun^3))
AU_OVER_RSUN = 215.03   # 1.495979e13 cm / 6.957e10 cm
R_EARTH_OVER_RSUN = 0.009168


def test_kepler_third_law_earth():
    # a sidereal year around a star of solar density is an orbit of 1 AU
    assert og.a_over_r(365.25636, RHO_SUN) == pytest.approx(AU_OVER_RSUN, rel=3e-3)


def test_earth_transit_duration():
    # a central transit of the Earth across the Sun lasts about 13 hours
    hours = og.t14(365.25, RHO_SUN, R_EARTH_OVER_RSUN, 0.0) * 24.0
    assert 12.9 < hours < 13.3


def test_small_angle_limit():
    # asin x -> x: T -> P (1 + k) / (pi a/R) for a wide orbit, b = 0
    for P, rho, k in ((300.0, 1.4, 0.01), (120.0, 0.7, 0.1), (50.0, 5.0, 0.0)):
        ar = og.a_over_r(P, rho)
        assert og.t14(P, rho, k, 0.0) == pytest.approx(P * (1 + k) / (np.pi * ar), rel=2e-4)


def test_impact_parameter_shortens_the_chord():
    # with sin i -> 1 the duration scales with the chord sqrt((1+k)^2 - b^2)
    P, rho = 200.0, 1.4
    full = og.t14(P, rho, 0.0, 0.0)
    assert og.t14(P, rho, 0.0, 0.6) == pytest.approx(0.8 * full, rel=1e-4)


def test_degenerate_orbits():
    assert og.t14(10.0, 1.4, 0.1, 1.2) == 0.0          # b beyond the limb: no transit
    assert og.t14(0.01, 1.4, 0.0, 0.0) == 0.005         # orbit inside the star: P / 2


def test_duration_limits_order():
    for P in (0.5, 3.0, 30.0, 300.0):
        lo, hi = og.duration_limits(P, 0.5, 3.0, 0.2, 0.9)
        assert 0 < lo < hi < P


@pytest.mark.parametrize("span,p_min,p_max,rho,os_", [(90.0, 0.5, 45.0, 1.41, 3.0), (730.5, 1.0, 400.0, 1.41, 2.0),
                                                      (27.4, 0.3, 13.7, 5.0, 5.0)])
def test_period_grid_meets_the_sampling_criterion(span, p_min, p_max, rho, os_):
    P = og.period_grid(span, p_min, p_max, rho, os_)
    assert np.all(np.diff(P) > 0)
    assert P[-1] == pytest.approx(p_max, rel=1e-14) and P[0] >= p_min
    f = 1.0 / (P * og.DAY_S)
    # one more step in f^(1/3) beyond the shortest period would pass p_min
    step = np.cbrt(f[0]) - np.cbrt(f[1])
    assert 1.0 / (np.cbrt(f[0]) + step) ** 3 / og.DAY_S < p_min
    # every step moves the last transit of the span by q / oversample of a phase
    df = f[:-1] - f[1:]
    fm = 0.5 * (f[:-1] + f[1:])
    ratio = df * span * og.DAY_S * os_ / og.duty_cycle(fm, rho)
    assert np.max(np.abs(ratio - 1.0)) < 2e-3


def test_period_grid_scaling():
    # the number of periods grows as oversample and as rho^(1/3)
    n = len(og.period_grid(90.0, 0.5, 45.0, 1.41, 3.0))
    assert len(og.period_grid(90.0, 0.5, 45.0, 1.41, 6.0)) == pytest.approx(2 * n, abs=2)
    assert len(og.period_grid(90.0, 0.5, 45.0, 8 * 1.41, 3.0)) == pytest.approx(2 * n, abs=2)


def test_keplerian_jrange_brute_force():
    rng = np.random.default_rng(4)
    periods = np.sort(rng.uniform(0.3, 60.0, 200))
    durations = np.geomspace(0.5, 15.0, 20) / 24.0
    jr = og.keplerian_jrange(periods, durations, 0.5, 3.0, 0.2, 0.9)
    for k, P in enumerate(periods):
        lo, hi = og.duration_limits(P, 0.5, 3.0, 0.2, 0.9)
        ok = [j for j, D in enumerate(durations) if lo <= D <= hi]
        if ok:
            assert (jr[k, 0], jr[k, 1]) == (ok[0], ok[-1])
        else:
            assert jr[k, 0] > jr[k, 1]
