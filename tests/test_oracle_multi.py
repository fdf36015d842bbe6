"""Pins of the single-event and iterative-search oracle (oracle/multi.py):
an exact template-matched single transit is the first event with its exact
depth (the Cauchy-Schwarz maximum of the likelihood ratio), the event list
obeys its own definition when checked by explicit loops, and the nulled
points of a signal are the grid points inside its transit windows counted
transit by transit."""

from fractions import Fraction as Fr

import numpy as np
import pytest

from synthlc import transit
from oracle import bruteforce as bf
from oracle import multi


def _curve(n, c, sig, rng):
    t = np.arange(n, dtype=np.float64) * c
    s = (sig * np.exp(0.3 * rng.normal(size=n))).astype(np.float32)
    return t, s


def test_exact_single_transit_is_the_first_event(ora):
    rng = np.random.default_rng(3)
    c = 297.3 / 86400
    n = 1000
    t, sig = _curve(n, c, 6e-4, rng)
    durs = np.array([0.8711, 1.9237, 3.1171]) / 24
    dense = transit.dense_template(1025)
    model = ora.template(dense, 256)
    g = ora.grid_plan(t[0], t[-1], c, durs, 256, t0_step=0.0613 * durs[0])
    bg = bf.BruteGrid(t[0], t[-1], c, durs, 256, t0_step=0.0613 * durs[0])
    jstar = 1
    istar = bg.I // 3
    A = 2.0 ** -9
    vec = A * bg.window_model(istar, jstar, model)
    f = vec[g.n_pad: g.n_pad + n].astype(np.float32)
    flux, ivar = ora.resample(g, t, f, sig)
    lin = ora.linear(g, flux, ivar, model)
    ev = multi.single_events(g, lin, 3)
    assert (ev[0]["epoch"], ev[0]["dur"]) == (istar, jstar)
    assert ev[0]["depth"] == pytest.approx(A, rel=1e-12)
    assert ev[0]["lr"] == pytest.approx(0.5 * np.sum(ivar * flux ** 2), rel=1e-11)
    # later events are pure zeros-and-noise-free windows: LR 0, not overlapping the first
    for e in ev[1:]:
        if e["epoch"] >= 0:
            assert abs(e["t0"] - ev[0]["t0"]) >= 0.5 * (e["duration"] + ev[0]["duration"])


def test_event_list_follows_its_definition(ora):
    rng = np.random.default_rng(8)
    c = 611.9 / 86400
    n = 600
    t, sig = _curve(n, c, 8e-4, rng)
    f = rng.normal(0.0, 8e-4, n).astype(np.float32)
    durs = np.array([1.1317, 2.5391]) / 24
    model = ora.template(transit.dense_template(257), 64)
    g = ora.grid_plan(t[0], t[-1], c, durs, 64, t0_step=0.1291 * durs[0])
    flux, ivar = ora.resample(g, t, f, sig)
    lin = ora.linear(g, flux, ivar, model)
    ev = multi.single_events(g, lin, 6)
    taken = []
    for e in ev:
        # explicit scan: the best admissible (j, i), first in (j, i) order on ties
        best, arg = -np.inf, None
        for j in range(g.n_dur):
            for i in range(g.n_t0):
                if not np.isfinite(lin["var"][j, i]):
                    continue
                ti = i * g.t0_step
                if any(abs(ti - tt) < 0.5 * (durs[j] + dd) for tt, dd in taken):
                    continue
                if lin["lr"][j, i] > best:
                    best, arg = lin["lr"][j, i], (j, i)
        assert (e["dur"], e["epoch"]) == arg
        taken.append((e["t0"], e["duration"]))
    lrs = [e["lr"] for e in ev]
    assert all(a >= b for a, b in zip(lrs, lrs[1:]))


@pytest.mark.parametrize("period,width", [(1.37, 1.5), (np.inf, 2.0), (0.61, 1.0)])
def test_mask_nulls_exactly_the_transit_windows(ora, period, width):
    c = 181.3 / 86400
    n = 2000
    t = np.arange(n) * c
    durs = np.array([1.5, 3.0]) / 24
    g = ora.grid_plan(t[0], t[-1], c, durs, 16)
    flux, ivar = ora.resample(g, t, np.ones(n, np.float32), np.full(n, 1e-3, np.float32))
    t0, D = 0.8123, 2.2 / 24
    mf, mi = multi.mask(g, flux, ivar, period, t0, D, width)
    # count transit by transit, in exact rationals
    cF, hw = Fr(g.cadence), Fr(width) * Fr(D) / 2
    centres = [Fr(t0)] if not np.isfinite(period) else \
        [Fr(t0) + m * Fr(period) for m in range(-int(3 / period) - 2, int(g.n * g.cadence / period) + 3)]
    want = set()
    for tc in centres:
        for q in range(g.n):
            if abs(q * cF - tc) <= hw:
                want.add(q)
    got = set(np.flatnonzero((mi == 0) & (ivar != 0)))
    assert got == {q for q in want if ivar[q] != 0}
    assert np.all(mf[list(want)] == 0)


def test_multi_template_ties_go_to_the_first():
    # two identical templates give identical searches: every period's
    # record is a tie, which the merge resolves to the first template
    from synthlc import workloads as W
    wl = W.tiny_single()
    sel = np.arange(0, len(wl.periods), 50)
    runs, win = multi.multi_template(wl, [wl.dense, wl.dense.copy()], sel=sel)
    assert np.array_equal(runs[0]["periodic"]["lr"], runs[1]["periodic"]["lr"])
    assert np.all(win[runs[0]["periodic"]["i"] >= 0] == 0)
