"""Parity metric between the GPU library and the FP64 oracle.

Relative error with a floor: err(x) = |x_gpu - x_ora| / max(|x_ora|, s_x).
The floors come from the absolute-value sums the oracle also returns
(aabs = sum w |f| m over the window, or over all transits for the fold):
  depth  s = aabs * var      (the size of the terms that cancel in S_fm)
  LR     s = |depth| * aabs / 2
  var    no floor (a sum of positive terms)
Plain relative error is ill-conditioned where S_fm is close to zero, i.e. in
pure-noise windows, which is why the floors exist.  The floors only bind
where the sum cancels: every element whose signed sum keeps at least half of
its absolute sum (|S_fm| >= aabs / 2, a cancellation factor of at most 2) is
also held to the plain relative error |x_gpu - x_ora| / |x_ora| <= TOL for
the depth and the LR (``well`` in the returned summaries counts them).

Near-ties: an argmax index mismatch is accepted only if the oracle's own
likelihood ratio at the GPU's choice is within TOL * max(LR*, floor) of the
oracle's maximum.
"""

from __future__ import annotations

import numpy as np

TOL = 1e-5


def rel(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def check_linear(depth, var, lr, ora: dict, tol: float = TOL) -> dict:
    """GPU public linear arrays vs oracle arrays of the same shape."""
    ok = np.isfinite(ora["var"])
    gok = np.isfinite(np.asarray(var))
    assert np.array_equal(ok, gok), f"null masks differ at {np.count_nonzero(ok != gok)} elements"
    assert np.all(np.isnan(np.asarray(depth)[~ok])) and np.all(np.asarray(lr)[~ok] == 0)
    d, v, l, a = ora["depth"][ok], ora["var"][ok], ora["lr"][ok], ora["aabs"][ok]
    e_d = rel(np.asarray(depth)[ok], d, a * v)
    e_v = rel(np.asarray(var)[ok], v)
    e_l = rel(np.asarray(lr)[ok], l, 0.5 * np.abs(d) * a)
    well = np.abs(d) / v >= 0.5 * a
    p_d = rel(np.asarray(depth)[ok][well], d[well])
    p_l = rel(np.asarray(lr)[ok][well], l[well])
    out = dict(depth=float(e_d.max(initial=0)), var=float(e_v.max(initial=0)), lr=float(e_l.max(initial=0)),
               n=int(ok.sum()), well=int(well.sum()), plain_depth=float(p_d.max(initial=0)),
               plain_lr=float(p_l.max(initial=0)),
               unfloored_frac=float(np.mean(rel(np.asarray(lr)[ok], l) <= tol)) if ok.any() else 1.0)
    assert out["depth"] <= tol and out["var"] <= tol and out["lr"] <= tol, out
    assert out["plain_depth"] <= tol and out["plain_lr"] <= tol, out
    return out


def check_periodic(gpu: dict, ora: dict, fold_at, periods, sel=None, tol: float = TOL) -> dict:
    """GPU per-period records vs oracle records.  ``fold_at(period, i, j)``
    evaluates one oracle candidate (for near-ties).  ``sel`` are the period
    indices the oracle evaluated (its arrays are in that order)."""
    g = {k: np.asarray(v) for k, v in gpu.items()}
    K = len(ora["lr"])
    sel = np.arange(K) if sel is None else np.asarray(sel)
    worst = dict(lr=0.0, depth=0.0, var=0.0)
    plain = dict(lr=0.0, depth=0.0)
    near_ties = 0
    well = 0
    for s in range(K):
        k = sel[s]
        oi, oj = int(ora["i"][s]), int(ora["j"][s])
        gi, gj = int(g["epoch"][k]), int(g["dur"][k])
        if oi < 0:
            assert gi < 0 and gj < 0 and g["lr"][k] == 0, f"period {k}: oracle null, GPU ({gi},{gj})"
            continue
        lr_o, z_o, zv_o, ab_o = ora["lr"][s], ora["z"][s], ora["zvar"][s], ora["aabs"][s]
        if (gi, gj) != (oi, oj):
            assert gi >= 0, f"period {k}: GPU null, oracle ({oi},{oj})"
            alt = fold_at(periods[k], gi, gj)
            assert alt is not None, f"period {k}: GPU chose a null candidate"
            floor = 0.5 * abs(z_o) * ab_o
            gap = (lr_o - alt[0]) / max(abs(lr_o), floor)
            assert gap <= tol, f"period {k}: GPU ({gi},{gj}) vs oracle ({oi},{oj}), LR gap {gap:.3g}"
            near_ties += 1
            lr_o, z_o, zv_o, ab_o = alt
        floor_l = 0.5 * abs(z_o) * ab_o
        worst["lr"] = max(worst["lr"], float(rel(g["lr"][k], lr_o, floor_l)))
        worst["depth"] = max(worst["depth"], float(rel(g["depth"][k], z_o, ab_o * zv_o)))
        worst["var"] = max(worst["var"], float(rel(g["depth_var"][k], zv_o)))
        if abs(z_o) / zv_o >= 0.5 * ab_o:  # well conditioned: plain relative error
            well += 1
            plain["lr"] = max(plain["lr"], float(rel(g["lr"][k], lr_o)))
            plain["depth"] = max(plain["depth"], float(rel(g["depth"][k], z_o)))
    assert max(worst.values()) <= tol, worst
    assert max(plain.values()) <= tol, plain
    worst["near_ties"] = near_ties
    worst["well"] = well
    worst["plain_lr"], worst["plain_depth"] = plain["lr"], plain["depth"]
    return worst
