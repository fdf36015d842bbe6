"""Period-recovery test of the paper's sensitivity comparison (Sec. 4.1,
Table 1), run on the GPU search.

Synthetic light curves of 173 d at 600-s cadence with a 7-d gap from day 90
carry one transit: period uniform over 1-86.5 d, duration uniform between
the period's Keplerian limits (circular orbits, stellar density 0.5-3
g/cm^3, k <= 0.2, b <= 0.9), depth log-uniform over 50-1000 ppm, the
default template's shape (b = 0.32), and white noise of 34, 160 or 800 ppm
per hour.  The search uses the paper's default grids: the optimally sampled
period grid for the span (solar density, oversampling 3) over 1-86.5 d,
24 log-spaced durations 0.6-30 h restricted per period to the same
Keplerian limits, and a reference-time step of 1% of the shortest duration.
A period is recovered when the best period lies within 1% of the injected
period, its half or its double.  Also reported: the Earth-analogue subset
(depth 75-125 ppm, period 58-87 d).

    python -m paper_2503_20875_amd.recovery --n 5000 --out recovery.json
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

SPAN_DAYS = 173.0
CADENCE_S = 600.0
GAP = (90.0, 97.0)
P_RANGE = (1.0, 86.5)
DEPTH_PPM = (50.0, 1000.0)
RHO = (0.5, 3.0)
K_MAX, B_MAX = 0.2, 0.9
NOISE_LEVELS = (34.0, 160.0, 800.0)  # ppm per hour
DURATIONS_H = (0.6, 30.0, 24)


def times() -> np.ndarray:
    """Observation times (days): 173 d at 600 s without the 7-d gap."""
    c = CADENCE_S / 86400.0
    t = np.arange(int(round(SPAN_DAYS / c)) + 1, dtype=np.float64) * c
    return t[(t < GAP[0]) | (t >= GAP[1])]


def noise_sigma(level_ppm_per_hour: float) -> float:
    """Per-point white-noise sigma (relative flux) whose one-hour mean has a
    standard deviation of the given ppm (reading T1): level * sqrt(1 h / cadence)."""
    return level_ppm_per_hour * 1e-6 * np.sqrt(3600.0 / CADENCE_S)


def recovered(found_period: float, true_period: float, tol: float = 0.01) -> bool:
    """The paper's recovery criterion (Sec. 4.1): the best period lies within
    1% of the injected period, its half or its double."""
    if not np.isfinite(found_period):
        return False
    return any(abs(found_period / (true_period * m) - 1.0) < tol for m in (1.0, 0.5, 2.0))


def draw(rng, limits, n: int):
    """n injections, one row (period, epoch, duration, depth) each: period
    uniform over 1-86.5 d, epoch uniform over one period, duration uniform
    between limits(P) = (shortest, longest) Keplerian duration (reading T2),
    depth log-uniform over 50-1000 ppm."""
    out = np.empty((n, 4))
    for r in range(n):
        P = rng.uniform(*P_RANGE)
        lo, hi = limits(P)
        out[r] = (P, rng.uniform(0.0, P), rng.uniform(lo, hi),
                  np.exp(rng.uniform(np.log(DEPTH_PPM[0]), np.log(DEPTH_PPM[1]))) * 1e-6)
    return out


def search_grids(cm, t):
    """The paper's default grids for this span: 24 log-spaced durations
    0.6-30 h, the optimally sampled period grid (solar density, oversampling
    3) over 1-86.5 d, and each period's Keplerian duration-index range."""
    durations = np.geomspace(DURATIONS_H[0] / 24.0, DURATIONS_H[1] / 24.0, DURATIONS_H[2])
    periods = cm.period_grid(t[-1] - t[0], P_RANGE[0], P_RANGE[1], cm.SOLAR_DENSITY, 3.0)
    jrange = cm.keplerian_jrange(periods, durations, RHO[0], RHO[1], K_MAX, B_MAX)
    return durations, periods, jrange


def light_curve(signal, level: float, rng):
    """(f, sigma) of one search input: the blocked-flux signal plus white
    noise of the level, as FP32 offsets from the baseline."""
    from synthlc import workloads as W
    sig = noise_sigma(level)
    y = 1.0 - signal + rng.normal(0.0, sig, signal.shape[0])
    return W.to_offset(y), np.full(signal.shape[0], sig, dtype=np.float32)


def run(n: int, seed: int = 20250405, levels=NOISE_LEVELS, batch: int = 256, log=None) -> dict:
    """n curves per noise level, searched `batch` curves at a time by the
    persistent batched search (every curve on the same time grid, period
    grid and Keplerian duration ranges).  The light curves are drawn in the
    same order as a curve-by-curve run would draw them, and batched records
    equal single-curve records, so the result does not depend on `batch`."""
    import torch
    import paper_2503_20875_amd as cm
    from synthlc import transit
    from synthlc import workloads as W
    t = times()
    dev = "cuda"
    cadence = CADENCE_S / 86400.0
    durations, periods, jrange = search_grids(cm, t)
    grid = cm.grid_plan(t[0], t[-1], cadence, durations, 0.0, 1024)
    model = cm.template_resample(torch.as_tensor(transit.dense_template(), device=dev), 1024)
    K = len(periods)
    inj = draw(np.random.default_rng(seed), lambda P: cm.duration_limits(P, RHO[0], RHO[1], K_MAX, B_MAX), n)
    cache = {}
    signals = [W.inject(t, W.Injection(period=p, epoch=e, duration=d, depth=dp), cache) for p, e, d, dp in inj]
    plans = {}

    def plan_for(m):
        if m not in plans:
            pl = cm.batch_plan([grid] * m, np.arange(m + 1) * t.shape[0], np.arange(m + 1) * K)
            plans[m] = (pl, cm.batch_workspace(pl),
                        torch.as_tensor(np.tile(t, m), device=dev), torch.as_tensor(np.tile(periods, m), device=dev),
                        torch.as_tensor(np.tile(jrange, (m, 1)), device=dev))
        return plans[m]

    results = {}
    t_gpu = 0.0
    for level in levels:
        rng = np.random.default_rng(seed + int(level))
        hit = np.zeros(n, dtype=bool)
        best_p = np.full(n, np.nan)
        for b0 in range(0, n, batch):
            rows = range(b0, min(n, b0 + batch))
            fs, ss = zip(*(light_curve(signals[r], level, rng) for r in rows))
            pl, work, t_d, p_d, jr_d = plan_for(len(rows))
            f_d = torch.as_tensor(np.concatenate(fs), device=dev)
            s_d = torch.as_tensor(np.concatenate(ss), device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = cm.batch_search(pl, t_d, f_d, s_d, model, p_d, work=work, jrange=jr_d)
            torch.cuda.synchronize()
            t_gpu += time.perf_counter() - t0
            if int(out["status"].item()) != 0 or not bool((out["done"] == 1).all()):
                raise RuntimeError(f"batched search status {int(out['status'].item())}")
            for r, b in zip(rows, cm.best_records(out["best"])):
                best_p[r] = b["period"] if b["k"] >= 0 else np.nan
                hit[r] = b["k"] >= 0 and recovered(b["period"], inj[r, 0])
            if log:
                log(f"{level:g} ppm/h: {rows[-1] + 1}/{n} searched, {hit[:rows[-1] + 1].sum()} recovered")
        earth = (inj[:, 3] >= 75e-6) & (inj[:, 3] <= 125e-6) & (inj[:, 0] >= 58.0) & (inj[:, 0] <= 87.0)
        results[f"{level:g}"] = {"n": n, "recovered": int(hit.sum()), "percent": 100.0 * hit.mean(),
                                 "earth_analogue_n": int(earth.sum()), "earth_analogue_recovered": int(hit[earth].sum())}
        if log:
            log(f"{level:g} ppm/h: {hit.sum()}/{n} recovered ({100.0 * hit.mean():.1f}%)")
    return {"n_per_level": n, "seed": seed, "n_periods": K, "n_durations": len(durations), "n_t0": int(grid.n_t0),
            "n_points": int(t.shape[0]), "batch": batch, "seconds_per_search": t_gpu / (n * len(levels)),
            "levels": results}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=1000, help="light curves per noise level")
    ap.add_argument("--seed", type=int, default=20250405)
    ap.add_argument("--batch", type=int, default=256, help="curves per batched search")
    ap.add_argument("--levels", default="",
                    help="comma-separated noise levels in ppm per hour (default: the paper's three)")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    levels = tuple(float(v) for v in a.levels.split(",")) if a.levels else NOISE_LEVELS
    import torch
    if not torch.cuda.is_available():
        print("recovery: no GPU", file=sys.stderr)
        return 2
    res = run(a.n, a.seed, levels=levels, batch=a.batch, log=lambda m: print(f"[recovery] {m}", flush=True))
    text = json.dumps(res)
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
