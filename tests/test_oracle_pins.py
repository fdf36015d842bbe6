"""Pins of the FP64 CPU oracle against things other than itself: closed forms
derived from the paper's equations, exact noiseless injections, special cases
that reduce to textbook statistics, an independent brute force on tiny
inputs, invariances, and the numbers the paper prints."""

import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from synthlc import transit, workloads as W
from oracle import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def tiny(ora):
    wl = W.tiny_single()
    return wl, ora.search(wl)


def _rel(a, b, floor=0.0):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


# ---------------------------------------------------------------- closed forms
def test_linear_lr_closed_form_and_nonnegative(tiny):
    """Eq. 2 evaluated at the ML depth equals Delta^2 / (2 var) (expand the
    square: sum w(D m f - D^2 m^2/2) with D = sum w f m / sum w m^2), which is
    >= 0 because the constant model is nested in the transit model."""
    _, r = tiny
    lin = r["linear"]
    ok = np.isfinite(lin["var"])
    assert ok.sum() > 0.5 * ok.size
    closed = 0.5 * lin["depth"][ok] ** 2 / lin["var"][ok]
    floor = 0.5 * np.abs(lin["depth"][ok]) * lin["aabs"][ok]
    assert np.max(_rel(lin["lr"][ok], closed, floor)) < 1e-9  # two-pass Eq. 2 cancels O(1) terms
    assert np.all(lin["lr"][ok] >= -1e-12 * floor)
    # nulls are encoded as documented
    assert np.all(np.isnan(lin["depth"][~ok])) and np.all(lin["lr"][~ok] == 0)


def test_periodic_lr_closed_form(tiny):
    """Summing Eq. 4 over transits at the inverse-variance common depth gives
    Z^2 / (2 var_Z) once each single-transit LR is Delta^2/(2 var)."""
    _, r = tiny
    p = r["periodic"]
    ok = p["i"] >= 0
    closed = 0.5 * p["z"][ok] ** 2 / p["zvar"][ok]
    floor = 0.5 * np.abs(p["z"][ok]) * p["aabs"][ok]
    assert np.max(_rel(p["lr"][ok], closed, floor)) < 1e-9
    assert np.all(p["lr"][ok] >= 0)


def test_long_period_reduces_to_linear(ora, tiny):
    """With a period longer than the whole reference-time span every epoch has
    a single transit, so the fold returns the linear search's global maximum
    (ties: smallest duration, then epoch)."""
    wl, r = tiny
    g = r["grid"]
    lin = r["linear"]
    span = g.n_t0 * g.t0_step
    per = ora.periodic(g, lin, np.array([span * 1.5, span * 3.0]))
    flat = lin["lr"].reshape(-1)
    jb, ib = divmod(int(np.argmax(flat)), g.n_t0)
    for s in range(2):
        assert per["i"][s] == ib and per["j"][s] == jb
        assert per["lr"][s] == pytest.approx(flat.max(), rel=1e-12)
        assert per["z"][s] == pytest.approx(lin["depth"][jb, ib], rel=1e-12)
        assert per["zvar"][s] == pytest.approx(lin["var"][jb, ib], rel=1e-12)


# ------------------------------------------------------- exact noiseless input
def _regular_curve(n, cadence, sigma, rng, lognormal=0.0):
    t = np.arange(n) * cadence + 1.25
    s = sigma * np.exp(lognormal * rng.normal(size=n))
    return t, s.astype(np.float32)


@pytest.mark.parametrize("seed", [3, 11])
def test_noiseless_injection_exact(ora, seed):
    """Flux equal to A times the sampled template on the windows of one
    periodic candidate (and zero elsewhere): every contributing window returns
    depth A exactly, the fold returns Z = A, LR = sum(w f^2)/2 (the
    Cauchy-Schwarz maximum over all candidates), so the search must pick that
    very candidate.  Template indices are computed in exact rationals."""
    rng = np.random.default_rng(seed)
    # irregular decimal parameters: no window edge or template cell boundary
    # falls exactly on a grid point, where FP64 evaluation (the oracle's
    # definition) and exact rationals may legitimately round differently
    c = 301.7 / 86400
    n = 900
    t, sig = _regular_curve(n, c, 5e-4, rng, lognormal=0.4)
    durs = np.array([0.9137, 1.7093, 2.6351]) / 24
    periods = np.sort(rng.uniform(0.55, 1.4, 9))
    dense = transit.dense_template(1025)
    model = ora.template(dense, 256)
    g = ora.grid_plan(t[0], t[-1], c, durs, 256, t0_step=0.0537 * durs[0])
    bg = bf.BruteGrid(t[0], t[-1], c, durs, 256, t0_step=0.0537 * durs[0])
    assert (bg.N, bg.I) == (g.n, g.n_t0)
    kstar, jstar = 4, 1
    P = periods[kstar]
    istar = int(rng.integers(0, bg.epochs_per_period(P)))
    A = 2.0 ** -10  # power of two: A * m is exact in FP32
    vec = np.zeros(bg.N)
    used = []
    for x in bg.transit_epochs(istar, P):
        gx = bg.window_model(x, jstar, model)
        if gx is not None:
            vec += A * gx
            used.append(x)
    assert len(used) >= 2
    # map the resampled-grid signal back onto the (regular) observations
    f = vec[g.n_pad: g.n_pad + n].astype(np.float32)
    assert np.array_equal(f.astype(np.float64), vec[g.n_pad: g.n_pad + n])
    flux, ivar = ora.resample(g, t, f, sig)
    lin = ora.linear(g, flux, ivar, model)
    for x in used:
        assert lin["depth"][jstar, x] == pytest.approx(A, rel=1e-12)
    per = ora.periodic(g, lin, periods)
    assert per["i"][kstar] == istar and per["j"][kstar] == jstar
    assert per["z"][kstar] == pytest.approx(A, rel=1e-12)
    bound = 0.5 * np.sum(ivar * flux ** 2)
    assert per["lr"][kstar] == pytest.approx(bound, rel=1e-11)
    assert ora.best(per) == kstar
    assert np.all(per["lr"] <= bound * (1 + 1e-11))


# ------------------------------------------------------- textbook special case
def test_box_template_uniform_sigma_is_arithmetic_mean(ora):
    """A one-sample (box) template with uniform sigma: the ML depth is the
    plain mean of the window fluxes, its variance sigma^2/L and the LR
    L mean^2 / (2 sigma^2) -- the statistic a box search uses with uniform
    errors (Sec. 3.1 contrasts this with the weighted mean)."""
    rng = np.random.default_rng(5)
    c = 613.3 / 86400  # irregular values: no window edge exactly on a grid point
    n = 700
    t = np.arange(n) * c
    sig = 8e-4
    f = rng.normal(0, sig, n).astype(np.float32)
    durs = np.array([1.0317, 2.4811]) / 24
    g = ora.grid_plan(t[0], t[-1], c, durs, 1, t0_step=0.1037 * durs[0])
    flux, ivar = ora.resample(g, t, f, np.full(n, sig, np.float32))
    lin = ora.linear(g, flux, ivar, np.array([1.0], np.float32))
    checked = 0
    for j, D in enumerate(durs):
        for i in range(0, g.n_t0, 7):
            ts = Fr(i) * Fr(g.t0_step) - Fr(float(D)) / 2
            te = ts + Fr(float(D))
            if ts < 0 or te > (g.n - 1) * Fr(c):
                assert np.isnan(lin["depth"][j, i])
                continue
            lo, hi = math.ceil(ts / Fr(c)), math.floor(te / Fr(c))
            pts = [q for q in range(lo, hi + 1) if ivar[q] > 0]
            if not pts:
                assert np.isnan(lin["depth"][j, i])
                continue
            vals = flux[pts]
            L = len(pts)
            s2 = 1.0 / ivar[pts[0]]
            assert lin["depth"][j, i] == pytest.approx(vals.mean(), rel=1e-9, abs=1e-15)
            assert lin["var"][j, i] == pytest.approx(s2 / L, rel=1e-12)
            assert lin["lr"][j, i] == pytest.approx(L * vals.mean() ** 2 / (2 * s2), rel=1e-8, abs=1e-14)
            checked += 1
    assert checked > 100


# ------------------------------------------------------------------ resampling
def test_resample_regular_is_identity_plus_padding(ora):
    rng = np.random.default_rng(0)
    c = 120.0 / 86400
    t = 3.0 + np.arange(500) * c
    f = rng.normal(0, 1e-3, 500).astype(np.float32)
    s = rng.uniform(5e-4, 2e-3, 500).astype(np.float32)
    g = ora.grid_plan(t[0], t[-1], c, np.array([0.05, 0.1]), 64)
    flux, ivar = ora.resample(g, t, f, s)
    assert g.n == 500 + 2 * g.n_pad and g.n_pad == math.ceil(0.05 / c)
    sl = slice(g.n_pad, g.n_pad + 500)
    assert np.allclose(flux[sl], f.astype(np.float64), rtol=1e-15, atol=0)  # (w f)/w to an ulp
    assert np.allclose(ivar[sl], 1.0 / s.astype(np.float64) ** 2, rtol=1e-15)
    assert np.all(ivar[: g.n_pad] == 0) and np.all(ivar[g.n_pad + 500:] == 0)


def test_resample_colocated_weighted_mean(ora):
    c = 0.01
    t = np.array([0.0, 0.1, 0.1004, 0.0996, 0.2, 0.3])
    f = np.array([1e-3, 2e-3, 4e-3, -1e-3, 0.0, 5e-4], np.float32)
    s = np.array([1e-3, 1e-3, 2e-3, 4e-3, 1e-3, 1e-3], np.float32)
    g = ora.grid_plan(t[0], t[-1], c, np.array([0.02]), 8)
    flux, ivar = ora.resample(g, t, f, s)
    q = g.n_pad + 10
    w = 1.0 / s[1:4].astype(np.float64) ** 2
    assert ivar[q] == pytest.approx(w.sum(), rel=1e-15)
    assert flux[q] == pytest.approx(np.sum(w * f[1:4]) / w.sum(), rel=1e-14)
    # formal uncertainty of a uniform-sigma mean is sigma / sqrt(k)
    assert 1 / math.sqrt(ivar[g.n_pad + 0]) == pytest.approx(1e-3, rel=1e-6)
    # empty points are null, missing data (nan, sigma <= 0) is skipped
    assert ivar[g.n_pad + 5] == 0 and flux[g.n_pad + 5] == 0
    f2 = f.copy(); f2[0] = np.nan
    s2 = s.copy(); s2[5] = 0
    flux2, ivar2 = ora.resample(g, t, f2, s2)
    assert ivar2[g.n_pad] == 0 and ivar2[g.n_pad + 30] == 0


def test_resample_permutation_invariant(ora):
    wl = W.small_random(7)
    g = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 64)
    a = ora.resample(g, wl.t, wl.f, wl.sigma)
    perm = np.random.default_rng(1).permutation(wl.n_obs)
    b = ora.resample(g, wl.t[perm], wl.f[perm], wl.sigma[perm])
    assert np.array_equal(a[1] > 0, b[1] > 0)
    assert np.allclose(a[0], b[0], rtol=1e-13, atol=1e-18)
    assert np.allclose(a[1], b[1], rtol=1e-13)


# ------------------------------------------------------------------ invariances
def test_scale_invariance(ora):
    """f, sigma -> a f, a sigma: depths scale by a, LR and SNR unchanged."""
    wl = W.small_random(2)
    a = 4.0  # power of two: the scaled FP32 inputs are exact
    r1 = ora.search(wl, t0_step=0.05 * wl.durations[0])
    wl2 = W.Workload(**{**wl.__dict__, "f": (wl.f * a).astype(np.float32),
                        "sigma": (wl.sigma * a).astype(np.float32)})
    r2 = ora.search(wl2, t0_step=0.05 * wl.durations[0])
    l1, l2 = r1["linear"], r2["linear"]
    ok = np.isfinite(l1["var"])
    assert np.allclose(l2["depth"][ok], a * l1["depth"][ok], rtol=1e-12, atol=1e-18)
    assert np.allclose(l2["lr"][ok], l1["lr"][ok], rtol=1e-9, atol=1e-12)
    p1, p2 = r1["periodic"], r2["periodic"]
    assert np.array_equal(p1["i"], p2["i"]) and np.array_equal(p1["j"], p2["j"])
    assert np.allclose(p2["lr"], p1["lr"], rtol=1e-9)


# ------------------------------------------------------------------ brute force
@pytest.mark.parametrize("seed", [1, 4])
def test_oracle_matches_bruteforce(ora, seed):
    """Every linear element and every period's best candidate agree with the
    exact-rational, full-likelihood brute force (exhaustive argmax)."""
    wl = W.small_random(seed, n_obs=260, n_dur=3, n_per=6, p_range=(0.5, 1.2), dur_h=(1.0, 3.0))
    step = 0.0813 * wl.durations[0]
    M = 128
    g = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, M, t0_step=step)
    bg = bf.BruteGrid(wl.t[0], wl.t[-1], wl.cadence, wl.durations, M, t0_step=step)
    assert (bg.N, bg.I, bg.n_pad) == (g.n, g.n_t0, g.n_pad)
    model = ora.template(wl.dense, M)
    flux, ivar = ora.resample(g, wl.t, wl.f, wl.sigma)
    bflux, bw = bg.resample(wl.t, wl.f, wl.sigma)
    assert np.array_equal(ivar > 0, bw > 0)
    assert np.allclose(flux, bflux, rtol=1e-13, atol=1e-18)
    assert np.allclose(ivar, bw, rtol=1e-13)
    lin = ora.linear(g, flux, ivar, model)
    windows = {}
    n_ok = 0
    for j in range(g.n_dur):
        for i in range(g.n_t0):
            gv = bg.window_model(i, j, model)
            windows[(i, j)] = gv
            r = None if gv is None else bf.fit(gv, bflux, bw)
            if r is None:
                assert np.isnan(lin["depth"][j, i]) and lin["lr"][j, i] == 0
                continue
            n_ok += 1
            fl = lin["aabs"][j, i]
            assert abs(lin["depth"][j, i] - r[0]) <= 1e-10 * max(abs(r[0]), fl / (1 / r[1]))
            assert lin["var"][j, i] == pytest.approx(r[1], rel=1e-12)
            assert abs(lin["lr"][j, i] - r[2]) <= 1e-8 * max(abs(r[2]), 0.5 * abs(r[0]) * fl)
    assert n_ok > 1000
    # windows of one period must not overlap for the fold to equal the fit
    assert np.all(wl.periods > 2 * wl.durations[-1])
    per = ora.periodic(g, lin, wl.periods)
    brute = bf.periodic(bg, bflux, bw, model, wl.periods, windows=windows)
    for k, b in enumerate(brute):
        assert b is not None
        assert (per["i"][k], per["j"][k]) == (b[1], b[2])
        assert per["lr"][k] == pytest.approx(b[0], rel=1e-8)
        assert per["z"][k] == pytest.approx(b[3], rel=1e-9)
        assert per["zvar"][k] == pytest.approx(b[4], rel=1e-12)


# ------------------------------------------------------------ paper's numbers
def test_template_nearest_neighbour_error_matches_fig1(ora):
    gv = golden()["nearest_neighbour_error"]
    tp = golden()["default_template"]
    dense = transit.dense_template(16385, tp["p"], tp["b"], tp["u1"], tp["u2"])
    M = gv["n_model"]
    model = ora.template(dense, M).astype(np.float64)
    tau = (np.arange(400000) + 0.5) / 400000
    truth = transit.shape_at(tau, dense)
    nn = model[np.minimum(M - 1, np.floor(tau * M).astype(int))]
    err = np.abs(nn - truth)
    assert 0.8 * gv["max_error"] <= err.max() <= 1.2 * gv["max_error"]
    assert gv["mean_error"] / 3 <= err.mean() <= 3 * gv["mean_error"]
    # fewer samples, larger error (Fig. 1 trend)
    m2 = ora.template(dense, 256).astype(np.float64)
    err2 = np.abs(m2[np.minimum(255, np.floor(tau * 256).astype(int))] - truth)
    assert err2.max() > 2 * err.max()


def test_template_linear_interpolation(ora):
    """Cell-centred samples of a linear ramp are exact; a constant stays constant."""
    ramp = np.linspace(0.0, 1.0, 1001)
    m = ora.template(ramp, 100).astype(np.float64)
    assert np.allclose(m, (np.arange(100) + 0.5) / 100, atol=1e-7)
    assert np.all(ora.template(np.ones(17), 33) == 1.0)


def test_paper_worked_example_period_and_aliases(ora):
    """Sec. 2.2 / Fig. 3 example: 5-d, 1000 ppm transits at 10, 30, 50 d peak
    at 20 d, with weaker peaks at the 10-d and 40-d aliases.  Unstated
    choices: 60-d span at 30-min cadence, white noise 300 ppm."""
    ex = golden()["worked_example"]
    rng = np.random.default_rng(8)
    c = 30.0 / 1440
    t = np.arange(0.0, 60.0, c)
    dense = transit.dense_template(2049)
    sig = np.zeros_like(t)
    for tc in ex["transit_times"]:
        sig += ex["depth"] * transit.shape_at((t - tc) / ex["duration"] + 0.5, dense)
    y = 1.0 - sig + rng.normal(0, 3e-4, t.shape[0])
    periods = np.geomspace(7.0, 48.0, 400)
    wl = W.Workload("example", t, W.to_offset(y), np.full(t.shape[0], 3e-4, np.float32), c,
                    np.array([2.5, 3.5, 5.0]), periods, dense, n_model=512)
    r = ora.search(wl, with_linear=False)
    lr = r["periodic"]["lr"]
    kb = r["best"]
    assert abs(periods[kb] / ex["true_period"] - 1) < golden()["recovery_criterion"]["rel_tol"]
    for alias in ex["aliases"]:
        near = np.abs(periods / alias - 1) < 0.02
        peak = lr[near].max()
        assert peak < lr[kb]
        # and it is a local peak: clearly above the periodogram 12% either side
        side = [lr[np.argmin(np.abs(periods - alias * f))] for f in (0.88, 1.12)]
        assert peak > 1.3 * max(side)


# ------------------------------------------------- zero-offset log-likelihood
def test_loglike0_matches_bruteforce_and_gaussian_density(ora):
    """l0 (Eq. 1 at zero depth over the non-null resampled points) equals the
    brute force's full Eq. 1 at depth 0, the sum of scipy's normal log
    densities N(flux; 0, w^-1/2), and l0 + LR of a window equals the full
    log-likelihood of that window's fitted model (Sec. 2.2: the LR is the
    difference of the two log-likelihoods)."""
    from scipy.stats import norm
    wl = W.small_random(2, n_obs=300, n_dur=2, n_per=3, dur_h=(1.0, 3.0))
    step = 0.0913 * wl.durations[0]
    M = 128
    g = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, M, t0_step=step)
    bg = bf.BruteGrid(wl.t[0], wl.t[-1], wl.cadence, wl.durations, M, t0_step=step)
    flux, ivar = ora.resample(g, wl.t, wl.f, wl.sigma)
    bflux, bw = bg.resample(wl.t, wl.f, wl.sigma)
    l0 = ora.loglike0(g, flux, ivar)
    zero = np.zeros(bg.N)
    assert l0 == pytest.approx(bf.loglike(zero, 0.0, bflux, bw), rel=1e-13)
    ok = ivar > 0
    assert ok.sum() < ok.size  # the padding and the gap are null points
    dens = float(np.sum(norm.logpdf(flux[ok], loc=0.0, scale=1.0 / np.sqrt(ivar[ok]))))
    assert l0 == pytest.approx(dens, rel=1e-13)
    model = ora.template(wl.dense, M)
    lin = ora.linear(g, flux, ivar, model)
    rng = np.random.default_rng(0)
    done = 0
    for _ in range(400):
        j, i = int(rng.integers(0, g.n_dur)), int(rng.integers(0, g.n_t0))
        gv = bg.window_model(i, j, model)
        if gv is None or not np.isfinite(lin["var"][j, i]):
            continue
        full = bf.loglike(gv, lin["depth"][j, i], bflux, bw)
        assert l0 + lin["lr"][j, i] == pytest.approx(full, rel=1e-12, abs=1e-9 * abs(l0))
        done += 1
    assert done > 100


def test_loglike0_uniform_sigma_closed_form(ora):
    """Uniform sigma, n non-null points: l0 = -sum f^2 / (2 sigma^2)
    - (n/2) ln(2 pi sigma^2)."""
    rng = np.random.default_rng(8)
    c = 120.0 / 86400.0
    t = np.arange(3000) * c + 1000.0
    t = np.delete(t, np.arange(700, 1100))  # a gap of null points
    sigma = 4e-4
    f = (rng.normal(0, sigma, t.size) + 1e-4).astype(np.float32)
    s = np.full(t.size, sigma, dtype=np.float32)
    g = ora.grid_plan(t[0], t[-1], c, [0.05, 0.1], 64)
    flux, ivar = ora.resample(g, t, f, s)
    s64 = float(np.float32(sigma))
    ff = f.astype(np.float64)
    expect = -0.5 * np.sum(ff ** 2) / s64 ** 2 - 0.5 * t.size * math.log(2 * math.pi * s64 ** 2)
    assert np.count_nonzero(ivar > 0) == t.size
    assert ora.loglike0(g, flux, ivar) == pytest.approx(expect, rel=1e-12)


# ------------------------------------------------------- edges of the period range
def test_period_range_edges(ora):
    """Reading for the period range: a period shorter than the reference-time
    step, or not finite, is not evaluated and gets the null record, even when
    some durations are shorter than it; a period of at least I steps has one
    transit per epoch, so its record is the best single window of the allowed
    durations; the brute force agrees on every evaluated period."""
    wl = W.small_random(5, n_obs=200, n_dur=3, n_per=4, p_range=(0.5, 1.0), dur_h=(0.6, 2.0))
    M = 64
    step = 1.7 * wl.durations[0]  # a step longer than the shortest duration
    g = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, M, t0_step=step)
    bg = bf.BruteGrid(wl.t[0], wl.t[-1], wl.cadence, wl.durations, M, t0_step=step)
    model = ora.template(wl.dense, M)
    flux, ivar = ora.resample(g, wl.t, wl.f, wl.sigma)
    lin = ora.linear(g, flux, ivar, model)
    span = g.n_t0 * g.t0_step
    short = [0.5 * step, step * (1 - 1e-9), 1.2 * wl.durations[0]]
    assert all(wl.durations[0] < p < step for p in short[1:])
    bad = [float("nan"), float("inf"), -1.0, 0.0]
    longp = [span * 1.0000001, span * 4.0, 1e30]
    periods = np.array(short + bad + [step] + longp)
    per = ora.periodic(g, lin, periods)
    for k in range(len(short) + len(bad)):
        assert per["i"][k] == -1 and per["j"][k] == -1 and per["lr"][k] == 0, periods[k]
        assert np.isnan(per["z"][k]) and per["zvar"][k] == np.inf
        assert ora.fold_at(g, lin, periods[k], 0, 0) is None
    n0 = len(short) + len(bad)
    # P = dt with D_0 < P: evaluated (one epoch, a transit at every reference time)
    assert per["i"][n0] == 0 and per["j"][n0] == 0
    # P >= I dt: the best single window among the durations shorter than P
    flat = lin["lr"].reshape(-1)
    jb, ib = divmod(int(np.argmax(flat)), g.n_t0)
    for k in range(n0 + 1, len(periods)):
        assert (per["i"][k], per["j"][k]) == (ib, jb)
        assert per["lr"][k] == pytest.approx(flat.max(), rel=1e-12)
    brute = bf.periodic(bg, *bg.resample(wl.t, wl.f, wl.sigma), model, periods[n0 + 1:n0 + 3])
    for k, b in enumerate(brute):
        assert (per["i"][n0 + 1 + k], per["j"][n0 + 1 + k]) == (b[1], b[2])
        assert per["lr"][n0 + 1 + k] == pytest.approx(b[0], rel=1e-8)
    assert bf.periodic(bg, *bg.resample(wl.t, wl.f, wl.sigma), model, periods[:2]) == [None, None]
