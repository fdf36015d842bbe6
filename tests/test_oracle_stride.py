"""Pins of the oracle's coarser, duration-scaled fold epoch grid (an option
the paper mentions adopting from TLS, Sec. 2.1.3): duration j evaluates only
the reference times that are multiples of its stride."""

from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import grids as og
from synthlc import workloads as W


@pytest.fixture(scope="module")
def ora():
    import oracle
    return oracle


def test_strides_follow_their_definition():
    """s_j * dt <= fraction * D_j < (s_j + 1) * dt in exact arithmetic (up
    to the rule's 1e-9 tolerance on whole multiples), and s_j >= 1."""
    durs = np.geomspace(0.5, 15.0, 20) / 24.0
    for frac in (0.01, 0.02, 0.005, 0.1):
        dt = 0.01 * durs[0]
        s = og.epoch_strides(durs, dt, frac)
        assert s.dtype == np.int32 and np.all(s >= 1)
        for D, sj in zip(durs, s):
            q = Fr(frac) * Fr(float(D)) / Fr(dt)
            if q >= 1:
                assert Fr(int(sj)) <= q + Fr(1, 10**8) and q < int(sj) + 1
            else:
                assert int(sj) == 1
    # whole multiples land on the multiple, not one short
    d0 = 1.0 / 24.0
    assert list(og.epoch_strides([d0, 2 * d0, 3 * d0, 7 * d0], 0.01 * d0, 0.01)) == [1, 2, 3, 7]


def test_unit_strides_are_the_plain_fold(ora):
    wl = W.tiny_single()
    r = ora.search(wl)
    g, lin = r["grid"], r["linear"]
    plain = ora.periodic(g, lin, wl.periods)
    ones = ora.periodic(g, lin, wl.periods, stride=np.ones(g.n_dur, dtype=np.int32))
    for k in plain:
        assert np.array_equal(plain[k], ones[k], equal_nan=True)


def test_strided_fold_is_the_plain_fold_on_a_subset(ora):
    """Each period's strided best is the best of the plain fold over the
    epochs kept: never above the plain best, equal to it when the plain
    winner is on the coarse grid, and its epoch a multiple of its stride."""
    wl = W.tiny_single()
    r = ora.search(wl)
    g, lin = r["grid"], r["linear"]
    st = np.array([1, 2, 3, 4, 5, 7, 9, 13][:g.n_dur], dtype=np.int32)
    plain = ora.periodic(g, lin, wl.periods)
    coarse = ora.periodic(g, lin, wl.periods, stride=st)
    n_same = 0
    for k in range(len(wl.periods)):
        if coarse["i"][k] < 0:
            continue
        j, i = coarse["j"][k], coarse["i"][k]
        assert i % st[j] == 0
        assert coarse["lr"][k] <= plain["lr"][k]
        if plain["i"][k] % st[plain["j"][k]] == 0:
            assert (i, j) == (plain["i"][k], plain["j"][k]) and coarse["lr"][k] == plain["lr"][k]
            n_same += 1
        alt = ora.fold_at(g, lin, wl.periods[k], i, j)
        assert alt[0] == coarse["lr"][k]
    assert 0 < n_same < len(wl.periods)


@pytest.mark.parametrize("seed", [2, 7])
def test_strided_oracle_matches_bruteforce(ora, seed):
    """Every period's strided best candidate agrees with the exact-rational,
    full-likelihood brute force restricted to the same epochs."""
    wl = W.small_random(seed, n_obs=260, n_dur=3, n_per=6, p_range=(0.5, 1.2), dur_h=(1.0, 3.0))
    step = 0.0813 * wl.durations[0]
    M = 128
    g = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, M, t0_step=step)
    bg = bf.BruteGrid(wl.t[0], wl.t[-1], wl.cadence, wl.durations, M, t0_step=step)
    model = ora.template(wl.dense, M)
    flux, ivar = ora.resample(g, wl.t, wl.f, wl.sigma)
    bflux, bw = bg.resample(wl.t, wl.f, wl.sigma)
    lin = ora.linear(g, flux, ivar, model)
    assert np.all(wl.periods > 2 * wl.durations[-1])
    st = np.array([2, 3, 5], dtype=np.int32)
    per = ora.periodic(g, lin, wl.periods, stride=st)
    brute = bf.periodic(bg, bflux, bw, model, wl.periods, stride=st)
    for k, b in enumerate(brute):
        assert b is not None
        assert (per["i"][k], per["j"][k]) == (b[1], b[2])
        assert per["lr"][k] == pytest.approx(b[0], rel=1e-8)
        assert per["z"][k] == pytest.approx(b[3], rel=1e-9)
        assert per["zvar"][k] == pytest.approx(b[4], rel=1e-12)


def test_bad_strides_are_rejected(ora):
    wl = W.tiny_single()
    r = ora.search(wl)
    with pytest.raises(ValueError):
        ora.periodic(r["grid"], r["linear"], wl.periods, stride=np.zeros(r["grid"].n_dur, dtype=np.int32))
    with pytest.raises(ValueError):
        ora.periodic(r["grid"], r["linear"], wl.periods, stride=np.ones(r["grid"].n_dur + 1, dtype=np.int32))
