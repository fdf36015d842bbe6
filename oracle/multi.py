"""Oracle for the single-event search and the iterative multi-signal search
-- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy on top of the oracle's own linear and periodic searches,
written from the definitions:

* Single transits are searched for in the linear-search output (Sec. 1,
  Sec. 5): event e is the candidate (j, i) with the largest likelihood ratio
  whose transit window does not overlap any earlier event's,
  |t_i - t_e| < (D_j + D_e) / 2 excluding it; ties go to the smallest j, then
  the smallest i.
* The multi-planet analysis of Sec. 5 searches again after nulling the flux
  in and around the strongest signal: a resampled point at time t (after the
  grid origin) is nulled when |t - t0 - n P| <= width * D / 2 for the nearest
  integer n (or |t - t0| for a single event).

Only the tests may import this module; it shares no code with the GPU
package.
"""

from __future__ import annotations

import numpy as np

import oracle


def single_events(g, lin: dict, n_events: int) -> list:
    """The n strongest non-overlapping single events of an oracle linear
    search (dicts with epoch, dur, t0, duration, lr, depth, depth_var, snr;
    epoch -1 once no candidate remains)."""
    lr = np.where(np.isfinite(lin["var"]), lin["lr"], -np.inf)
    J, I = lr.shape
    t = np.arange(I, dtype=np.float64) * g.t0_step
    durs = g.durations_array
    free = np.isfinite(lin["var"]).copy()
    out = []
    for _ in range(n_events):
        masked = np.where(free, lr, -np.inf)
        flat = int(np.argmax(masked))  # first maximum in (j, i) order
        if not np.isfinite(masked.reshape(-1)[flat]):
            out.append(dict(epoch=-1, dur=-1, t0=np.nan, duration=np.nan, lr=0.0, depth=np.nan,
                            depth_var=np.inf, snr=0.0))
            continue
        j, i = divmod(flat, I)
        ev = dict(epoch=i, dur=j, t0=i * g.t0_step, duration=durs[j], lr=lr[j, i], depth=lin["depth"][j, i],
                  depth_var=lin["var"][j, i])
        ev["snr"] = ev["depth"] / np.sqrt(ev["depth_var"])
        out.append(ev)
        for jj in range(J):
            free[jj] &= ~(np.abs(t - ev["t0"]) < 0.5 * (durs[jj] + ev["duration"]))
    return out


def mask(g, flux, ivar, period: float, t0: float, duration: float, width: float):
    """Copies of (flux, ivar) with the signal's transits nulled."""
    flux = np.array(flux, dtype=np.float64)
    ivar = np.array(ivar, dtype=np.float64)
    tq = np.arange(g.n, dtype=np.float64) * g.cadence
    d = tq - t0
    if np.isfinite(period) and period > 0:
        d = d - np.floor(d / period + 0.5) * period
    hit = np.abs(d) <= 0.5 * width * duration
    flux[hit] = 0.0
    ivar[hit] = 0.0
    return flux, ivar


def iterative(wl, n_signals: int, width: float = 1.5, sel=None):
    """Search, null the best periodic signal, search again; per pass the
    oracle's grid, linear arrays, periodic records and best index.  Periods
    are restricted to `sel` (indices) when given."""
    g = oracle.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model)
    model = oracle.template(wl.dense, wl.n_model)
    flux, ivar = oracle.resample(g, wl.t, wl.f, wl.sigma)
    periods = np.asarray(wl.periods, dtype=np.float64)
    sel = np.arange(len(periods)) if sel is None else np.asarray(sel)
    passes = []
    for _ in range(n_signals):
        lin = oracle.linear(g, flux, ivar, model)
        per = oracle.periodic(g, lin, periods, sel=sel)
        kb = oracle.best(per)
        passes.append(dict(grid=g, linear=lin, periodic=per, best=kb, flux=flux, ivar=ivar))
        if kb < 0:
            break
        k = sel[kb]
        j = per["j"][kb]
        flux, ivar = mask(g, flux, ivar, periods[k], per["i"][kb] * g.t0_step, g.durations_array[j], width)
    return passes


def multi_template(wl, denses, sel=None):
    """One oracle search per template on the same light curve, merged per
    period: the largest likelihood ratio, ties to the earlier template; a
    null record (epoch -1) never wins over a valid one."""
    runs = []
    for dense in denses:
        w2 = type(wl)(**{**wl.__dict__, "dense": dense})
        runs.append(oracle.search(w2, sel=sel))
    per = [r["periodic"] for r in runs]
    K = len(per[0]["lr"])
    win = np.full(K, -1, dtype=np.int64)
    for k in range(K):
        for s_, p in enumerate(per):
            if p["i"][k] < 0:
                continue
            if win[k] < 0 or p["lr"][k] > per[win[k]]["lr"][k]:
                win[k] = s_
    return runs, win
