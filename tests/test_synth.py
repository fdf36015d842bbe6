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


def test_learned_curves_device_generator_recipe():
    """The device generator of the learned workload (run here on the CPU
    device) follows the recipe: 80 000 points at 2 min, gaps as NaN sigma,
    log-normal sigma around 800 ppm, injections inside the stated ranges,
    and the injected signal added with the template's shape."""
    import numpy as np
    import torch
    from synthlc import workloads as W
    gen = W.LearnedCurves(5, device="cpu")
    n_planet = 0
    for _ in range(12):
        t, f, s, injs = gen.draw()
        assert t.shape == f.shape == s.shape == (W.LEARNED_N_POINTS,)
        assert f.dtype == torch.float32 and s.dtype == torch.float32 and t.dtype == torch.float64
        assert abs(float(t[1] - t[0]) * 86400.0 - 120.0) < 1e-6
        ok = torch.isfinite(s)
        ls = torch.log(s[ok].double() / 800e-6)
        assert abs(float(ls.mean())) < 0.01 and abs(float(ls.std()) - 0.25) < 0.01
        gap_days = float((~ok).sum()) * 120.0 / 86400.0
        assert gap_days < 20.0
        for inj in injs:
            n_planet += 1
            assert 1.0 <= inj.period <= 100.0 and 50e-6 <= inj.depth <= 3000e-6 and 0.0 <= inj.b <= 0.9
            assert inj.duration > 0
            # the mean offset inside transits exceeds the mean outside by a
            # fraction of the depth set by the limb-darkened shape
            phase = np.mod(t.numpy() - inj.epoch + 0.5 * inj.period, inj.period) - 0.5 * inj.period
            inside = np.abs(phase) < 0.25 * inj.duration
            if inside.sum() > 200:
                d = float(f.numpy()[inside].mean() - f.numpy()[~inside].mean())
                assert 0.5 * inj.depth < d < 1.2 * inj.depth + 5 * 800e-6 / np.sqrt(inside.sum())
    assert n_planet >= 3


def test_survey_subset_process_pool_gives_the_same_curves():
    """Each survey curve has its own seed, so generating them in a forked
    pool returns the serial curves, in order."""
    serial = W.survey_subset(24, n_min=5000, n_max=9000)
    seen = []
    pooled = W.survey_subset(24, n_min=5000, n_max=9000, workers=3, progress=seen.append)
    assert seen == []  # progress is reported every 256 curves
    assert [c.name for c in pooled] == [c.name for c in serial]
    for a, b in zip(serial, pooled):
        for x, y in ((a.t, b.t), (a.f, b.f), (a.sigma, b.sigma), (a.periods, b.periods)):
            assert np.array_equal(x, y)
        assert a.injections == b.injections
