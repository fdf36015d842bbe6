"""Pins of the input generators (transit shape, workloads) against textbook
geometry and the workload recipes."""

import math

import numpy as np
import pytest

from synthlc import transit, workloads as W


@pytest.mark.parametrize("z", [0.0, 0.3, 0.95, 0.975, 0.99, 1.0, 1.01, 1.02, 1.029])
def test_uniform_disc_blocked_fraction_is_lens_area(z):
    """With no limb darkening the blocked fraction is the two-circle overlap
    area divided by pi; at full overlap it is p^2."""
    p = 0.03
    got = transit.blocked_fraction(z, p, 0.0, 0.0)
    assert got == pytest.approx(transit.overlap_area(z, p) / math.pi, rel=1e-8, abs=1e-14)
    if z <= 1 - p:
        assert got == pytest.approx(p * p, rel=1e-10)


def test_large_planet_covering_centre():
    """z < p (planet disc covers the stellar centre) uses the full-circle branch."""
    p = 0.4
    for z in (0.0, 0.1, 0.35, 0.8):
        got = transit.blocked_fraction(z, p, 0.0, 0.0)
        assert got == pytest.approx(transit.overlap_area(z, p) / math.pi, rel=1e-8)


def test_limb_darkening_normalisation():
    """The intensity integrates to pi (1 - u1/3 - u2/6) over the disc, and a
    small planet at disc centre hides p^2 I(0) / that."""
    u1, u2 = 0.4804, 0.1867
    x, w = np.polynomial.legendre.leggauss(200)
    phi = np.pi / 4 * (x + 1)  # r = sin(phi) makes mu = cos(phi) smooth
    rr = np.sin(phi)
    num = np.sum(np.pi / 4 * w * transit.intensity(rr, u1, u2) * 2 * np.pi * rr * np.cos(phi))
    assert num == pytest.approx(transit.stellar_flux(u1, u2), rel=1e-9)
    p = 1e-3
    centre = transit.blocked_fraction(0.0, p, u1, u2)
    assert centre == pytest.approx(p * p / (1 - u1 / 3 - u2 / 6), rel=1e-5)


def test_dense_template_shape():
    d = transit.dense_template(2049)
    assert d.max() == 1.0
    assert d[0] == pytest.approx(0.0, abs=1e-12) and d[-1] == pytest.approx(0.0, abs=1e-12)
    assert np.allclose(d, d[::-1], atol=1e-12)          # symmetric chord
    mid = d.shape[0] // 2
    assert np.all(np.diff(d[: mid + 1]) >= -1e-15)      # monotone ingress
    # grazing chords are V-shaped: shallower plateau relative to the peak
    g = transit.dense_template(2049, b=0.99)
    assert np.mean(g) < np.mean(d)


def test_workload_recipes():
    wl = W.tiny_single()
    assert wl.n_obs == 19728 - 2 * 720
    assert wl.f.dtype == np.float32 and wl.sigma.dtype == np.float32 and wl.t.dtype == np.float64
    assert np.all(np.diff(wl.t) > 0)
    assert wl.durations.shape == (8,) and wl.periods.shape == (1000,)
    assert np.allclose(np.diff(1 / wl.periods[::-1]), np.diff(1 / wl.periods[::-1])[0])
    assert wl.durations[0] == pytest.approx(0.5 / 24) and wl.durations[-1] == pytest.approx(6 / 24)
    # seeded: identical on regeneration
    assert np.array_equal(W.tiny_single().f, wl.f)


def test_transit_duration_sun_like():
    """Earth around the Sun: ~13 h central transit."""
    d = transit.transit_duration_days(365.25, 0.0, p=0.009)
    assert 12.5 / 24 < d < 13.5 / 24
