"""Pins of the FP64 proposal-network oracle: gradients against central finite
differences, and the lag correlation against a direct double loop."""

import numpy as np
import pytest

from oracle import net


def small_case(seed=0, B=2, C=3, L=48, width=5, n_event=2, hidden=6):
    rng = np.random.default_rng(seed)
    p = net.init_params(c_in=C, width=width, n_layers=5, n_event=n_event, hidden=hidden, seed=seed)
    for k in p:  # non-zero biases so every term is exercised
        if k.startswith("b") or k in ("p", "u"):
            p[k] = rng.normal(0, 0.1, p[k].shape)
    x = rng.uniform(0, 1, (B, C, L))
    lo = np.array([2, 3, 5, 9, 14])
    hi = np.array([2, 4, 8, 13, 21])
    q = (np.arange(5) + 0.5) / 5
    y = np.zeros((B, 5))
    y[0, 2] = 1
    return p, x, lo, hi, q, y


def total_loss(p, x, lo, hi, q, y):
    z = net.forward(p, x, lo, hi, q)
    return net.bce_loss(z, y, pos_weight=4.0)[0]


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    p, x, lo, hi, q, y = small_case(seed)
    z, cache = net.forward(p, x, lo, hi, q, keep=True)
    _, gz = net.bce_loss(z, y, pos_weight=4.0)
    g = net.backward(p, cache, gz, lo, hi)
    rng = np.random.default_rng(seed + 10)
    h = 1e-6
    for name in list(p.keys()) + ["x"]:
        arr = x if name == "x" else p[name]
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = total_loss(p, x, lo, hi, q, y)
            flat[idx] = old - h
            lm = total_loss(p, x, lo, hi, q, y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            # relu kinks and max ties are measure-zero with random inputs
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, idx, fd, an)


def test_lag_correlation_direct():
    rng = np.random.default_rng(3)
    e = rng.uniform(0, 1, (2, 3, 40))
    lags = np.array([1, 4, 7, 39, 40])
    a = net.lag_correlation(e, lags)
    for b in range(2):
        for c in range(3):
            for i, tau in enumerate(lags):
                ref = sum(e[b, c, t] * e[b, c, t + tau] for t in range(40 - tau)) / 40 if tau < 40 else 0.0
                assert a[b, c, i] == pytest.approx(ref, abs=1e-14)


def test_periodic_events_peak_at_their_spacing():
    """A train of events every 37 bins correlates most at lag 37."""
    e = np.zeros((1, 1, 400))
    e[0, 0, 5::37] = 1.0
    lags = np.arange(1, 120)
    a = net.lag_correlation(e, lags)[0, 0]
    assert lags[np.argmax(a)] == 37
    assert a[lags == 74][0] > 0 and a[lags == 20][0] == 0


def test_windows_cover_the_lag_axis():
    lo, hi, q, edges = net.windows_for(512, 1.0, 100.0, 111.5 / 8192)
    assert lo.shape == (512,) and np.all(hi >= lo) and np.all(np.diff(lo) >= 0)
    assert lo[0] == round(1.0 / (111.5 / 8192)) and hi[-1] == round(100.0 / (111.5 / 8192))
    p = net.init_params()
    assert 150_000 < net.n_params(p) < 260_000


def test_bf16_rounding_known_values():
    """Round-to-nearest-even onto the 8-bit significand: exact values pass,
    halfway cases go to the even neighbour."""
    one_ulp = 2.0 ** -7  # spacing of bfloat16 in [1, 2)
    vals = np.array([1.0, 1.0 + one_ulp, 1.0 + one_ulp / 2, 1.0 + 3 * one_ulp / 2, -2.5, 3.0e38, 1.0e-30])
    got = net.bf16(vals)
    assert got[0] == 1.0 and got[1] == 1.0 + one_ulp
    assert got[2] == 1.0  # tie -> even (1.0)
    assert got[3] == 1.0 + 2 * one_ulp  # tie -> even
    assert got[4] == -2.5
    assert abs(got[5] - 3.0e38) / 3.0e38 < 2 ** -8 and abs(got[6] - 1e-30) / 1e-30 < 2 ** -8
    x = np.random.default_rng(0).normal(size=1000)
    r = net.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)
    assert np.array_equal(net.bf16(r), r)


def test_bf16_trunk_gradients_consistent():
    """With the trunk rounded to bfloat16, the head and projection gradients
    still match central differences (rounding is piecewise constant, so only
    the parameters after the trunk are differentiated here)."""
    p, x, lo, hi, q, y = small_case(4)
    z, cache = net.forward(p, x, lo, hi, q, keep=True, bf16_trunk=True)
    _, gz = net.bce_loss(z, y, pos_weight=4.0)
    g = net.backward(p, cache, gz, lo, hi)
    h = 1e-6
    for name in ("P", "p", "U", "u", "v", "v0"):
        flat = p[name].reshape(-1)
        for idx in range(min(4, flat.size)):
            old = flat[idx]
            flat[idx] = old + h
            lp = net.bce_loss(net.forward(p, x, lo, hi, q, bf16_trunk=True), y, 4.0)[0]
            flat[idx] = old - h
            lm = net.bce_loss(net.forward(p, x, lo, hi, q, bf16_trunk=True), y, 4.0)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, idx)


def test_standardise_zero_mean_unit_variance_and_affine_invariant():
    rng = np.random.default_rng(8)
    a = rng.normal(size=(2, 3, 50)) * 1e-3 + 5e-3
    n, sd = net.standardise(a)
    assert np.allclose(n.mean(axis=2), 0, atol=1e-12) and np.allclose((n * n).mean(axis=2), 1, atol=1e-5)
    n2, _ = net.standardise(7.0 * a - 3.0)
    assert np.allclose(n2, n, atol=1e-5)
    # constant input: no signal, output zero
    n0, _ = net.standardise(np.full((1, 1, 10), 0.25))
    assert np.all(n0 == 0)


def test_fold_pool_recovers_a_period():
    """Spikes every 10 bins starting at bin 3: the trial of 10 bins peaks at
    phase 3 with score n / sqrt(n) = sqrt(10); a detuned trial scores less."""
    e = np.zeros((1, 1, 100))
    e[0, 0, 3::10] = 1.0
    trials = np.array([[9.37, 10.0]])
    g, arg = net.fold_pool(e, trials)
    assert arg[0, 0, 0].tolist() == [1, 3]
    assert g[0, 0, 0] == pytest.approx(np.sqrt(10.0), abs=1e-12)
    g9, _ = net.fold_pool(e, trials[:, :1])
    assert g9[0, 0, 0] < np.sqrt(10.0)


def test_fold_offsets_are_nearest_multiples():
    """The fixed-point transit offsets equal round-half-up of k T, exactly
    (Fraction arithmetic on the FP64 trial)."""
    from fractions import Fraction
    rng = np.random.default_rng(4)
    for T in rng.uniform(1.0, 300.0, 20):
        R = net.fold_step(T)
        assert abs(Fraction(R, 2 ** 32) - Fraction(T)) <= Fraction(1, 2 ** 33)
        for k in range(0, 60, 7):
            assert ((k * R + 2 ** 31) >> 32) == int(np.floor(Fraction(k * R, 2 ** 32) + Fraction(1, 2)))


def test_fold_trials_inside_windows():
    lo, hi, q, edges = net.windows_for(32, 1.0, 100.0, 0.05)
    t = net.fold_trials(edges, 4, 0.05)
    assert t.shape == (32, 4)
    assert np.all(t * 0.05 > edges[:-1, None]) and np.all(t * 0.05 < edges[1:, None])
    assert np.all(np.diff(t, axis=1) > 0)


@pytest.mark.parametrize("seed", [0, 3])
def test_fold_pool_gradients_match_central_differences(seed):
    rng = np.random.default_rng(seed)
    B, C, L, W = 2, 3, 60, 5
    p = net.init_params(c_in=C, width=5, n_layers=5, n_event=2, hidden=6, seed=seed, fold=True)
    for k in p:
        if k.startswith("b") or k in ("p", "u"):
            p[k] = rng.normal(0, 0.1, p[k].shape)
    x = rng.uniform(0, 1, (B, C, L))
    edges = np.geomspace(2.0, 20.0, W + 1)
    trials = net.fold_trials(edges, 3, 1.0)
    lo = hi = np.zeros(W, dtype=np.int64)
    q = (np.arange(W) + 0.5) / W
    y = np.zeros((B, W))
    y[0, 1] = y[1, 3] = 1
    z, cache = net.forward(p, x, lo, hi, q, keep=True, trials=trials)
    _, gz = net.bce_loss(z, y, pos_weight=3.0)
    g = net.backward(p, cache, gz, lo, hi)
    h = 1e-6
    for name in list(p.keys()) + ["x"]:
        arr = x if name == "x" else p[name]
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, min(5, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = net.bce_loss(net.forward(p, x, lo, hi, q, trials=trials), y, 3.0)[0]
            flat[idx] = old - h
            lm = net.bce_loss(net.forward(p, x, lo, hi, q, trials=trials), y, 3.0)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, idx, fd)
