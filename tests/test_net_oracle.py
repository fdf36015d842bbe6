"""Pins of the FP64 proposal-network oracle: gradients against central finite
differences, the fold pooling against closed cases and exact arithmetic, and
the bfloat16 rounding against its definition."""

import numpy as np
import pytest

from oracle import net


def small_case(seed=0, B=2, C=3, L=60, width=5, n_event=2, hidden=6, W=5):
    rng = np.random.default_rng(seed)
    p = net.init_params(c_in=C, width=width, n_layers=5, n_event=n_event, hidden=hidden, seed=seed)
    for k in p:  # non-zero biases so every term is exercised
        if k.startswith("b") or k in ("p", "u"):
            p[k] = rng.normal(0, 0.1, p[k].shape)
    x = rng.uniform(0, 1, (B, C, L))
    edges = np.geomspace(2.0, 20.0, W + 1)
    trials = net.fold_trials(edges, 3, 1.0)
    q = (np.arange(W) + 0.5) / W
    y = np.zeros((B, W))
    y[0, 1] = y[1, 3] = 1
    return p, x, q, trials, y


def total_loss(p, x, q, trials, y, **kw):
    return net.bce_loss(net.forward(p, x, q, trials, **kw), y, 3.0)[0]


@pytest.mark.parametrize("seed", [0, 3])
def test_gradients_match_central_differences(seed):
    p, x, q, trials, y = small_case(seed)
    z, cache = net.forward(p, x, q, trials, keep=True)
    _, gz = net.bce_loss(z, y, pos_weight=3.0)
    g = net.backward(p, cache, gz)
    rng = np.random.default_rng(seed + 10)
    h = 1e-6
    for name in list(p.keys()) + ["x"]:
        arr = x if name == "x" else p[name]
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, min(5, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = total_loss(p, x, q, trials, y)
            flat[idx] = old - h
            lm = total_loss(p, x, q, trials, y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            # relu kinks and max ties are measure-zero with random inputs
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, idx, fd, an)


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


def test_fold_pool_brute_force():
    """Every (trial, phase) score written out with a direct loop over exact
    rational transit positions; the maximum, its first position and the
    runner-up agree, and a trial shorter than one bin is skipped."""
    from fractions import Fraction
    rng = np.random.default_rng(6)
    e = rng.normal(size=(1, 2, 47))
    trials = np.array([[3.3, 4.71, 0.5], [11.05, 12.9, 13.4]])
    g, arg, second = net.fold_pool(e, trials, runner_up=True)
    for w in range(2):
        for c in range(2):
            scores = []
            for s_, T in enumerate(trials[w]):
                if T < 1.0:
                    continue
                R = Fraction(net.fold_step(T), 2 ** 32)
                for ph in range(min(47, int(np.ceil(float(R))))):
                    pos = []
                    k = 0
                    while True:
                        x = ph + int(np.floor(k * R + Fraction(1, 2)))
                        if x >= 47:
                            break
                        pos.append(x)
                        k += 1
                    scores.append((sum(e[0, c, pos]) / np.sqrt(len(pos)), s_, ph))
            best = max(t[0] for t in scores)
            assert g[0, w, c] == pytest.approx(best, abs=1e-12)
            first = next(t for t in scores if t[0] == best)
            assert arg[0, w, c].tolist() == [first[1], first[2]]
            assert second[0, w, c] == pytest.approx(sorted(t[0] for t in scores)[-2], abs=1e-12)


def test_fold_pool_decides_in_fp32():
    """Two phases whose scores differ below FP32 resolution tie, and the tie
    goes to the first phase; a difference FP32 resolves decides.  The
    feature is the FP64 score of the winner."""
    e = np.zeros((1, 1, 4))
    e[0, 0, 0] = 1.0
    e[0, 0, 2] = 1.0 + 1e-12         # later phase, FP64-larger, FP32-equal
    trials = np.array([[4.0]])          # one transit per phase, n = 1
    g, arg = net.fold_pool(e, trials)
    assert arg[0, 0, 0].tolist() == [0, 0] and g[0, 0, 0] == 1.0
    e[0, 0, 2] = 1.0 + 2.0 ** -20       # resolved in FP32
    g, arg = net.fold_pool(e, trials)
    assert arg[0, 0, 0].tolist() == [0, 2] and g[0, 0, 0] == 1.0 + 2.0 ** -20
    # the FP32 score rounds the reciprocal square root once from FP64
    assert net.score32(3.0, 7) == np.float32(3.0) * np.float32(1.0 / np.sqrt(7.0))


def test_downsample_signed_keeps_the_sign():
    """Signed input on hand-made pairs: per bin the largest S_fm/sqrt(S_mm)
    with its sign, null elements skipped, an all-null bin 0, clipping at
    +-30 before the division by 8; the |SNR| input of the same pairs is the
    bin's largest absolute value."""
    fold = np.zeros((1, 6, 2))
    fold[0, :, 0] = [-2.0, -8.0, 3.0, 1.0, 0.0, -1e4]
    fold[0, :, 1] = [4.0, 16.0, 9.0, 0.0, 0.0, 1.0]
    x = net.downsample_signed(fold, 3)       # bins {0,1}, {2,3}, {4,5}
    assert x[:, 0].tolist() == [-1.0 / 8.0, 1.0 / 8.0, -30.0 / 8.0]
    fold[0, 4:, 1] = 0.0                     # the last bin all null
    assert net.downsample_signed(fold, 3)[2, 0] == 0.0
    assert net.downsample(fold, 3)[:, 0].tolist() == [2.0 / 8.0, 1.0 / 8.0, 0.0]


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
    q, edges = net.windows_for(32, 1.0, 100.0)
    t = net.fold_trials(edges, 4, 0.05)
    assert t.shape == (32, 4)
    assert np.all(t * 0.05 > edges[:-1, None]) and np.all(t * 0.05 < edges[1:, None])
    assert np.all(np.diff(t, axis=1) > 0)
    assert edges[0] == 1.0 and edges[-1] == pytest.approx(100.0) and np.all(np.diff(edges) > 0)
    assert np.allclose(q, (np.arange(32) + 0.5) / 32)


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
    p, x, q, trials, y = small_case(4)
    z, cache = net.forward(p, x, q, trials, keep=True, bf16_trunk=True)
    _, gz = net.bce_loss(z, y, pos_weight=3.0)
    g = net.backward(p, cache, gz)
    h = 1e-6
    for name in ("P", "p", "U", "u", "v", "v0"):
        flat = p[name].reshape(-1)
        for idx in range(min(4, flat.size)):
            old = flat[idx]
            flat[idx] = old + h
            lp = total_loss(p, x, q, trials, y, bf16_trunk=True)
            flat[idx] = old - h
            lm = total_loss(p, x, q, trials, y, bf16_trunk=True)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, idx)


def test_parameter_count():
    """5 conv layers (16 -> 64, then 64 -> 64, 9 taps, biases), projection
    64 -> 8, head 9 -> 64 -> 1."""
    conv = 64 * 16 * 9 + 64 + 4 * (64 * 64 * 9 + 64)
    head = 8 * 64 + 8 + 64 * 9 + 64 + 64 + 1
    assert net.n_params(net.init_params()) == conv + head


def test_downsample_is_binned_single_event_snr(ora):
    """The network input (reading N1) pinned against the linear search: on a
    small curve the oracle's own depth and variance give the single-event SNR
    |depth| / sqrt(var) of every element; the maximum over each bin, clipped at
    30 and divided by 8, equals net.downsample of the (S_fm, S_mm) pairs
    (S_fm = depth / var, S_mm = 1 / var).  Bins follow floor(b I / L), so a
    bin count that does not divide I leaves ragged bins."""
    from synthlc import workloads as W
    wl = W.small_random(3, n_obs=400, n_dur=3)
    g = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 128, t0_step=0.05 * wl.durations[0])
    flux, ivar = ora.resample(g, wl.t, wl.f, wl.sigma)
    lin = ora.linear(g, flux, ivar, ora.template(wl.dense, 128))
    ok = np.isfinite(lin["var"])
    assert 0 < ok.sum() < ok.size
    pairs = np.zeros((g.n_dur, g.n_t0, 2))
    pairs[..., 0][ok] = lin["depth"][ok] / lin["var"][ok]
    pairs[..., 1][ok] = 1.0 / lin["var"][ok]
    for L in (7, 64, g.n_t0):
        got = net.downsample(pairs, L)
        for j in range(g.n_dur):
            for b in range(L):
                i0, i1 = (b * g.n_t0) // L, ((b + 1) * g.n_t0) // L
                vals = [abs(lin["depth"][j, i]) / np.sqrt(lin["var"][j, i]) for i in range(i0, i1) if ok[j, i]]
                expect = min(max(vals, default=0.0), 30.0) / 8.0
                assert got[b, j] == pytest.approx(expect, rel=1e-12, abs=1e-300)


def test_downsample_saturation_and_nulls():
    """A huge SNR saturates at 30 / 8 = 3.75; an all-null bin is 0; the sign
    of S_fm does not matter (a brightening is as strong as a dip)."""
    fold = np.zeros((2, 10, 2))
    fold[0, :, 0] = 1e6
    fold[0, :, 1] = 1.0
    fold[1, 5, :] = (-3.0, 1.0)   # SNR 3 in the second bin of duration 1
    out = net.downsample(fold, 2)
    assert np.array_equal(out[:, 0], [3.75, 3.75])
    assert out[0, 1] == 0.0 and out[1, 1] == pytest.approx(3.0 / 8.0)


def test_fold_phase_counts_follow_the_split_rule():
    """The rule the fold-pooling kernel applies instead of counting: with
    step R, phase 0 has n0 = (2^32 L - 2^31 - 1) // R + 1 positions inside a
    series of L bins, and every phase below n_ph = min(L, ceil(R / 2^32))
    has n0 of them below ph_split = L - (((n0 - 1) R + 2^31) >> 32) and
    n0 - 1 from there on.  Checked against counting every phase's positions
    (offsets by their definition), for random and edge-case trials."""
    rng = np.random.default_rng(11)
    cases = [(int(L), float(T)) for L, T in zip(rng.integers(1, 8193, 60), rng.uniform(1.0, 400.0, 60))]
    cases += [(int(L), float(L) * f) for L, f in zip(rng.integers(1, 8193, 30), rng.uniform(0.05, 3.0, 30))]
    cases += [(8192, 1.0), (8192, 1.5), (8192, 64.0), (8192, 1024.0), (8192, 8191.5), (8192, 8192.0), (8192, 1e9 - 1),
              (1, 1.0), (1, 7.3), (2, 1.0), (100, 99.9999), (100, 100.0), (100, 33.3333333)]
    for L, T in cases:
        R = net.fold_step(T)
        n_ph = min(L, -(-R // 2 ** 32))
        offs = []
        k = 0
        while (k * R + 2 ** 31) >> 32 < L:
            offs.append((k * R + 2 ** 31) >> 32)
            k += 1
        offs = np.array(offs, dtype=np.int64)
        counts = np.searchsorted(offs, L - np.arange(n_ph), side="left")  # positions ph + o < L
        n0 = (2 ** 32 * L - 2 ** 31 - 1) // R + 1
        ph_split = L - (((n0 - 1) * R + 2 ** 31) >> 32)
        assert n0 == len(offs) == counts[0], (L, T)
        want = np.where(np.arange(n_ph) < ph_split, n0, n0 - 1)
        assert np.array_equal(counts, want), (L, T)
        assert counts.min() >= 1
