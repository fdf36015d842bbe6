"""Seeded synthetic light curves and search grids.

Every workload here is an *input* to the transit search: observation times
(FP64 days), flux offsets from baseline (FP32; 0 = baseline, 1 = star fully
blocked, Sec. 2 units convention), per-point uncertainties (FP32), a dense
template, trial durations and trial periods.  Normalised fluxes y are made in
FP64 and converted once to offsets f = 1 - y, rounded to FP32, so every
consumer of a workload sees exactly the same FP32 arrays.

The workloads stand in for the paper's data (TESS/PLATO-like cadences and
baselines, Sec. 3.2 and Sec. 4); none of the paper's data sets is used.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import transit

DAY_S = 86400.0
HOUR = 1.0 / 24.0


@dataclasses.dataclass
class Injection:
    period: float          # days (np.inf for a single event)
    epoch: float           # mid-transit time of one transit (days)
    duration: float        # first-to-last contact (days)
    depth: float           # maximum flux offset
    b: float = transit.DEFAULT_B


@dataclasses.dataclass
class Workload:
    name: str
    t: np.ndarray          # float64 [n_obs], ascending
    f: np.ndarray          # float32 [n_obs], flux offset from baseline
    sigma: np.ndarray      # float32 [n_obs]
    cadence: float         # resample cadence (days)
    durations: np.ndarray  # float64 [J], ascending (days)
    periods: np.ndarray    # float64 [K], ascending (days)
    dense: np.ndarray      # float64 dense template, max 1
    n_model: int = 1024    # template samples M
    t0_step_frac: float = 0.01
    injections: List[Injection] = dataclasses.field(default_factory=list)
    seed: int = 0

    @property
    def n_obs(self) -> int:
        return int(self.t.shape[0])


def to_offset(y: np.ndarray) -> np.ndarray:
    """FP64 normalised flux -> FP32 offset from baseline (single rounding)."""
    return (1.0 - np.asarray(y, dtype=np.float64)).astype(np.float32)


def inject(t: np.ndarray, inj: Injection, dense_cache: Optional[dict] = None) -> np.ndarray:
    """Blocked-flux signal (>= 0) of a periodic transit at times t."""
    key = round(inj.b, 6)
    if dense_cache is not None and key in dense_cache:
        dense = dense_cache[key]
    else:
        dense = transit.dense_template(b=inj.b)
        if dense_cache is not None:
            dense_cache[key] = dense
    if np.isfinite(inj.period):
        phase = np.mod(t - inj.epoch + 0.5 * inj.period, inj.period) - 0.5 * inj.period
    else:
        phase = t - inj.epoch
    tau = phase / inj.duration + 0.5
    return inj.depth * transit.shape_at(tau, dense)


def random_gaps(rng, t_lo: float, t_hi: float, n_gaps: int, length: float,
                max_tries: int = 10000):
    """Start times of ``n_gaps`` non-overlapping gaps of fixed length."""
    starts: List[float] = []
    tries = 0
    while len(starts) < n_gaps:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place gaps")
        s = rng.uniform(t_lo, t_hi - length)
        if all(abs(s - o) >= length for o in starts):
            starts.append(s)
    return sorted(starts)


def uniform_frequency_periods(p_min: float, p_max: float, k: int) -> np.ndarray:
    freq = np.linspace(1.0 / p_max, 1.0 / p_min, k)
    return np.sort(1.0 / freq)


def log_periods(p_min: float, p_max: float, k: int) -> np.ndarray:
    return np.geomspace(p_min, p_max, k)


def log_durations(d_min_h: float, d_max_h: float, j: int) -> np.ndarray:
    return np.geomspace(d_min_h * HOUR, d_max_h * HOUR, j)


def running_median(y: np.ndarray, window: int) -> np.ndarray:
    """Centred running median (pandas' skip-list rolling median)."""
    import pandas as pd
    s = pd.Series(y)
    return s.rolling(window, center=True, min_periods=1).median().to_numpy()


def tiny_single(seed: int = 20250326) -> Workload:
    """One 27.4-d light curve at 2-min cadence (about one TESS sector):
    white noise 1000 ppm, two random 1-d gaps, one injected transit
    P = 5.3 d, depth 2000 ppm, duration 3 h.  8 log-spaced durations
    0.5-6 h; 1000 periods uniform in frequency over 1-13 d."""
    rng = np.random.default_rng(seed)
    c = 120.0 / DAY_S
    n = int(round(27.4 / c))
    t = np.arange(n, dtype=np.float64) * c
    keep = np.ones(n, dtype=bool)
    for s in random_gaps(rng, 0.0, t[-1], 2, 1.0):
        keep &= ~((t >= s) & (t < s + 1.0))
    t = t[keep]
    sig = 1000e-6
    inj = Injection(period=5.3, epoch=rng.uniform(0.0, 5.3), duration=3.0 * HOUR,
                    depth=2000e-6)
    y = 1.0 - inject(t, inj) + rng.normal(0.0, sig, t.shape[0])
    return Workload(
        name="single-lc 27.4d@120s (tiny)", t=t, f=to_offset(y),
        sigma=np.full(t.shape[0], sig, dtype=np.float32), cadence=c,
        durations=log_durations(0.5, 6.0, 8),
        periods=uniform_frequency_periods(1.0, 13.0, 1000),
        dense=transit.dense_template(), injections=[inj], seed=seed)


def tiny_two_planets(seed: int = 20250330) -> Workload:
    """The tiny light curve with two planets: 27.4 d at 2-min cadence, white
    noise 1000 ppm, two random 1-d gaps; P = 5.3 d / 2000 ppm / 3 h and
    P = 2.1 d / 1500 ppm / 2 h at random epochs.  8 log-spaced durations
    0.5-6 h; 1000 periods uniform in frequency over 1-13 d."""
    rng = np.random.default_rng(seed)
    c = 120.0 / DAY_S
    n = int(round(27.4 / c))
    t = np.arange(n, dtype=np.float64) * c
    keep = np.ones(n, dtype=bool)
    for s in random_gaps(rng, 0.0, t[-1], 2, 1.0):
        keep &= ~((t >= s) & (t < s + 1.0))
    t = t[keep]
    sig = 1000e-6
    injs = [Injection(period=5.3, epoch=rng.uniform(0.0, 5.3), duration=3.0 * HOUR, depth=2000e-6),
            Injection(period=2.1, epoch=rng.uniform(0.0, 2.1), duration=2.0 * HOUR, depth=1500e-6)]
    y = 1.0 - sum(inject(t, i) for i in injs) + rng.normal(0.0, sig, t.shape[0])
    return Workload(
        name="two-planet 27.4d@120s (tiny)", t=t, f=to_offset(y),
        sigma=np.full(t.shape[0], sig, dtype=np.float32), cadence=c,
        durations=log_durations(0.5, 6.0, 8),
        periods=uniform_frequency_periods(1.0, 13.0, 1000),
        dense=transit.dense_template(), injections=injs, seed=seed)


def high_cadence(seed: int = 20250327) -> Workload:
    """One 90-d light curve at 20-s cadence (TESS-20s-like): AR(1) red noise
    (phi = 0.9, marginal 300 ppm) plus 500 ppm white noise, pre-whitened by a
    centred 1-d running median over valid points; 5% of points masked as six
    0.75-d gaps; per-point sigma = 1.4826 * MAD of the pre-whitened flux.
    Transits P = 17.1 d / 400 ppm / 4 h and P = 3.2 d / 250 ppm / 1.5 h.
    20 log-spaced durations 0.5-15 h; 50 000 log-spaced periods 0.5-45 d."""
    rng = np.random.default_rng(seed)
    c = 20.0 / DAY_S
    n = int(round(90.0 / c))
    t = np.arange(n, dtype=np.float64) * c
    phi, marg = 0.9, 300e-6
    innov = marg * np.sqrt(1.0 - phi * phi)
    e = rng.normal(0.0, innov, n)
    red = np.empty(n)
    red[0] = rng.normal(0.0, marg)
    # AR(1) recursion via a linear filter
    from scipy.signal import lfilter
    red[1:] = lfilter([1.0], [1.0, -phi], e[1:], zi=[phi * red[0]])[0]
    white = rng.normal(0.0, 500e-6, n)
    keep = np.ones(n, dtype=bool)
    for s in random_gaps(rng, 0.0, t[-1], 6, 0.75):
        keep &= ~((t >= s) & (t < s + 0.75))
    injs = [Injection(17.1, rng.uniform(0.0, 17.1), 4.0 * HOUR, 400e-6),
            Injection(3.2, rng.uniform(0.0, 3.2), 1.5 * HOUR, 250e-6)]
    sig_blocked = sum(inject(t, inj) for inj in injs)
    y = 1.0 - sig_blocked + red + white
    t, y = t[keep], y[keep]
    trend = running_median(y, int(round(1.0 / c)))
    y = y - trend + 1.0
    resid = y - 1.0
    mad = np.median(np.abs(resid - np.median(resid)))
    sig = 1.4826 * mad
    return Workload(
        name="single-lc 90d@20s (high cadence)", t=t, f=to_offset(y),
        sigma=np.full(t.shape[0], sig, dtype=np.float32), cadence=c,
        durations=log_durations(0.5, 15.0, 20),
        periods=log_periods(0.5, 45.0, 50000),
        dense=transit.dense_template(), injections=injs, seed=seed)


def small_random(seed: int, n_obs: int = 600, cadence_s: float = 611.7,
                 n_dur: int = 3, n_per: int = 12, jitter: float = 0.3,
                 dup_frac: float = 0.1, gap_frac: float = 0.15,
                 sigma_lognorm: float = 0.3, depth: float = 3e-3,
                 p_range=(0.6, 2.5), dur_h=(1.0, 4.0)) -> Workload:
    """Small irregular light curve for exhaustive checks: jittered cadence,
    some co-located observations, gaps, lognormal per-point sigma and one
    injected transit."""
    rng = np.random.default_rng(seed)
    c = cadence_s / DAY_S
    t = np.arange(n_obs, dtype=np.float64) * c + rng.uniform(-jitter, jitter, n_obs) * c
    n_dup = int(dup_frac * n_obs)
    if n_dup:
        extra = t[rng.integers(0, n_obs, n_dup)] + rng.uniform(-0.2, 0.2, n_dup) * c
        t = np.concatenate([t, extra])
    t = np.sort(t) + rng.uniform(0.0, 3.0)
    n_tot = t.shape[0]
    if gap_frac > 0:
        g0 = rng.uniform(t[0], t[-1])
        glen = gap_frac * (t[-1] - t[0])
        keep = ~((t >= g0) & (t < g0 + glen))
        t = t[keep]
        n_tot = t.shape[0]
    sig = (1e-3 * np.exp(sigma_lognorm * rng.normal(size=n_tot))).astype(np.float32)
    per = rng.uniform(*p_range)
    inj = Injection(per, t[0] + rng.uniform(0.0, per), rng.uniform(*dur_h) * HOUR, depth)
    y = 1.0 - inject(t, inj) + rng.normal(size=n_tot) * sig.astype(np.float64)
    # irregular factors keep window edges off exact grid coincidences
    durs = log_durations(dur_h[0] * 0.7137, dur_h[1] * 1.2113, n_dur)
    pers = np.sort(rng.uniform(p_range[0] * 0.8, p_range[1] * 1.5, n_per))
    return Workload(name=f"small-random-{seed}", t=t, f=to_offset(y), sigma=sig,
                    cadence=c, durations=durs, periods=pers,
                    dense=transit.dense_template(), n_model=1024,
                    injections=[inj], seed=seed)


def duty_cycle_periods(p_min: float, p_max: float, span: float, d_min: float, alpha: float = 0.389):
    """Period grid with relative step dP/P = alpha * D_min / T (the phase
    shift of the last transit stays a fixed fraction of the shortest
    duration)."""
    step = alpha * d_min / span
    k = int(np.floor(np.log(p_max / p_min) / np.log1p(step))) + 1
    return p_min * (1.0 + step) ** np.arange(k)


def survey_curve(rng, n_points: int, cadence_s: float = 120.0, sigma_ppm: float = 800.0,
                 planet_frac: float = 0.3, durations=None, p_range=(0.5, 40.0), depth_range=(100e-6, 5000e-6),
                 b_step: float = 0.0):
    """One light curve of a batched survey: regular cadence, Poisson(1.5)
    gaps of U(0.2, 2) d, per-point sigma log-normal (log-sd 0.25) around
    sigma_ppm, and with probability planet_frac one transit with P log-uniform
    over p_range, depth log-uniform over depth_range (default 100-5000 ppm),
    b uniform 0-0.9 and the duration of a circular orbit around a
    Sun-density star.  b_step > 0 rounds b to that step (so the transit
    shapes of many curves come from a small cache)."""
    c = cadence_s / DAY_S
    t = np.arange(n_points, dtype=np.float64) * c
    span = t[-1]
    keep = np.ones(n_points, dtype=bool)
    for _ in range(rng.poisson(1.5)):
        glen = rng.uniform(0.2, 2.0)
        g0 = rng.uniform(0.0, max(span - glen, 1e-9))
        keep &= ~((t >= g0) & (t < g0 + glen))
    if keep.sum() < 2:
        keep[:2] = True
    t = t[keep]
    sig = sigma_ppm * 1e-6 * np.exp(0.25 * rng.normal(size=t.shape[0]))
    injs = []
    y = 1.0 + rng.normal(size=t.shape[0]) * sig
    if rng.uniform() < planet_frac:
        P = float(np.exp(rng.uniform(np.log(p_range[0]), np.log(p_range[1]))))
        b = float(rng.uniform(0.0, 0.9))
        if b_step > 0:
            b = round(round(b / b_step) * b_step, 6)
        dur = transit.transit_duration_days(P, b)
        inj = Injection(P, rng.uniform(0.0, P), dur,
                        float(np.exp(rng.uniform(np.log(depth_range[0]), np.log(depth_range[1])))), b)
        y = y - inject(t, inj)
        injs.append(inj)
    return t, to_offset(y), sig.astype(np.float32), injs


def batched_survey(n_curves: int, seed: int = 20250328, n_min: int = 5000, n_max: int = 120000,
                   n_dur: int = 16, d_min_h: float = 0.5, d_max_h: float = 10.0, alpha: float = 0.389,
                   p_min: float = 0.5, p_max: float = 40.0):
    """A batch of survey light curves of uneven length (uniform n_min-n_max
    points at 2-min cadence), shared durations, and per-curve duty-cycle
    period grids over [p_min, min(p_max, T/2)]."""
    rng = np.random.default_rng(seed)
    durs = log_durations(d_min_h, d_max_h, n_dur)
    curves = []
    for _ in range(n_curves):
        n = int(rng.integers(n_min, n_max + 1))
        t, f, s, injs = survey_curve(rng, n, durations=durs, p_range=(p_min, p_max))
        span = t[-1] - t[0]
        hi = min(p_max, span / 2.0)
        periods = duty_cycle_periods(p_min, hi, span, durs[0], alpha) if hi > p_min else np.zeros(0)
        curves.append(Workload(name=f"survey-{len(curves)}", t=t, f=f, sigma=s, cadence=120.0 / DAY_S,
                               durations=durs, periods=periods, dense=transit.dense_template(),
                               injections=injs, seed=seed))
    return curves


def _survey_member(args) -> Workload:
    """Curve k of a survey_subset (module level so a process pool can run it)."""
    k, n_curves, seed, n_min, n_max, durs, alpha, p_min, p_max = args
    rng = np.random.default_rng(seed + k)
    n = int(round(n_min + (k + 0.5) / n_curves * (n_max - n_min)))
    t, f, s, injs = survey_curve(rng, n, durations=durs, p_range=(p_min, p_max))
    span = t[-1] - t[0]
    hi = min(p_max, span / 2.0)
    periods = duty_cycle_periods(p_min, hi, span, durs[0], alpha) if hi > p_min else np.zeros(0)
    return Workload(name=f"survey-{k}", t=t, f=f, sigma=s, cadence=120.0 / DAY_S,
                    durations=durs, periods=periods, dense=transit.dense_template(),
                    injections=injs, seed=seed + k)


def survey_subset(n_curves: int, seed: int = 20250328, n_min: int = 5000, n_max: int = 120000,
                  n_dur: int = 16, d_min_h: float = 0.5, d_max_h: float = 10.0, alpha: float = 0.389,
                  p_min: float = 0.5, p_max: float = 40.0, workers: int = 1, progress=None):
    """A length-stratified stand-in for a large batched survey: curve k has
    the k-th of n_curves equal-probability strata of the uniform length
    distribution over [n_min, n_max] points (its stratum's midpoint), and its
    own generator seeded with seed + k; everything else as batched_survey.
    workers > 1 generates in a forked process pool (same curves: each has its
    own seed); progress(k_done) is called after every 256 curves."""
    durs = log_durations(d_min_h, d_max_h, n_dur)
    jobs = [(k, n_curves, seed, n_min, n_max, durs, alpha, p_min, p_max) for k in range(n_curves)]
    curves = []

    def take(it):
        for c in it:
            curves.append(c)
            if progress is not None and len(curves) % 256 == 0:
                progress(len(curves))

    if workers > 1:
        import multiprocessing
        with multiprocessing.get_context("fork").Pool(workers) as pool:
            take(pool.imap(_survey_member, jobs, chunksize=16))
    else:
        take(map(_survey_member, jobs))
    return curves


def long_baseline(seed: int = 20250329) -> Workload:
    """Earth analogue: one 730.5-d light curve at 25-s cadence (2 524 608
    points, PLATO-like), white noise 200 ppm per point, no gaps.  One transit
    signal P = 365.25 d, depth 100 ppm, duration 13 h, its epoch drawn so that
    both transits fall inside the data.  30 log-spaced durations 1-20 h;
    400 000 duty-cycle periods over 1-400 d (alpha = 0.263)."""
    rng = np.random.default_rng(seed)
    c = 25.0 / DAY_S
    n = int(round(730.5 / c))
    t = np.arange(n, dtype=np.float64) * c
    sig = 200e-6
    inj = Injection(period=365.25, epoch=rng.uniform(1.0, t[-1] - 365.25 - 1.0), duration=13.0 * HOUR,
                    depth=100e-6)
    y = 1.0 - inject(t, inj) + rng.normal(0.0, sig, n)
    durs = log_durations(1.0, 20.0, 30)
    return Workload(
        name="earth-analogue 730.5d@25s (long baseline)", t=t, f=to_offset(y),
        sigma=np.full(n, sig, dtype=np.float32), cadence=c, durations=durs,
        periods=duty_cycle_periods(1.0, 400.0, t[-1], durs[0], alpha=0.263),
        dense=transit.dense_template(), injections=[inj], seed=seed)


WORKLOADS = {
    "tiny": tiny_single,
    "high_cadence": high_cadence,
    "long_baseline": long_baseline,
}


# Learned-proposal workload: 80 000 points at 2-min cadence (111.1 d), noise
# and gaps as the batched survey, half the curves with one planet (P
# log-uniform 1-100 d, depth log-uniform 50-3000 ppm), 16 durations 0.5-10 h,
# plain period grid alpha = 0.389 over 1-100 d.
LEARNED_N_POINTS = 80000
LEARNED_DURATIONS_H = (0.5, 10.0, 16)
LEARNED_P_RANGE = (1.0, 100.0)


def learned_curve(rng):
    """One curve of the learned-proposal workload: (t, f, sigma, injections)."""
    return survey_curve(rng, LEARNED_N_POINTS, planet_frac=0.5, p_range=LEARNED_P_RANGE,
                        depth_range=(50e-6, 3000e-6), b_step=0.01)


def learned_grid():
    """Durations (days) and the plain period grid of the learned workload."""
    durations = log_durations(*LEARNED_DURATIONS_H)
    span = (LEARNED_N_POINTS - 1) * 120.0 / DAY_S
    periods = duty_cycle_periods(LEARNED_P_RANGE[0], LEARNED_P_RANGE[1], span, durations[0])
    return durations, periods


# Long-baseline proposal workload: curves of the Earth-analogue set-up (730.5 d
# at 25 s, white noise 200 ppm per point, 30 durations 1-20 h, 399 404
# periods 1-400 d), half with one planet (P log-uniform 1-400 d, depth
# log-uniform 20-400 ppm, b uniform 0-0.9 rounded to 0.01, circular orbit
# around a Sun-density star).  Generated on the GPU: 2.5 M points per curve.
LONG_P_RANGE = (1.0, 400.0)
LONG_DEPTH_RANGE = (20e-6, 400e-6)
LONG_SIGMA = 200e-6


def long_grid():
    """Durations (days) and periods of the long-baseline workload."""
    wl = long_baseline_shape()
    return wl["durations"], wl["periods"]


def long_baseline_shape():
    c = 25.0 / DAY_S
    n = int(round(730.5 / c))
    span = (n - 1) * c
    durs = log_durations(1.0, 20.0, 30)
    return dict(n=n, cadence=c, span=span, durations=durs,
                periods=duty_cycle_periods(1.0, 400.0, span, durs[0], alpha=0.263))


class LongCurves:
    """Light curves of the long-baseline proposal workload, generated on a
    torch device: the time grid is shared, the noise comes from a seeded
    device generator and the injection parameters from a seeded numpy
    generator.  draw() returns device (t, f, sigma) and the injections."""

    def __init__(self, seed: int, device="cuda", planet_frac: float = 0.5):
        import torch
        sh = long_baseline_shape()
        self.n, self.cadence = sh["n"], sh["cadence"]
        self.torch = torch
        self.device = device
        self.t = torch.arange(self.n, dtype=torch.float64, device=device) * self.cadence
        self.sigma = torch.full((self.n,), LONG_SIGMA, dtype=torch.float32, device=device)
        self.rng = np.random.default_rng(seed)
        self.gen = torch.Generator(device=device)
        self.gen.manual_seed(int(seed))
        self.planet_frac = planet_frac
        self.dense = {}

    def _dense(self, b: float):
        if b not in self.dense:
            self.dense[b] = self.torch.as_tensor(transit.dense_template(b=b), device=self.device)
        return self.dense[b]

    def draw(self):
        torch = self.torch
        off = -LONG_SIGMA * torch.randn(self.n, generator=self.gen, dtype=torch.float64, device=self.device)
        injs = []
        if self.rng.uniform() < self.planet_frac:
            P = float(np.exp(self.rng.uniform(np.log(LONG_P_RANGE[0]), np.log(LONG_P_RANGE[1]))))
            b = round(round(float(self.rng.uniform(0.0, 0.9)) / 0.01) * 0.01, 6)
            dur = transit.transit_duration_days(P, b)
            depth = float(np.exp(self.rng.uniform(np.log(LONG_DEPTH_RANGE[0]), np.log(LONG_DEPTH_RANGE[1]))))
            inj = Injection(P, float(self.rng.uniform(0.0, P)), dur, depth, b)
            dense = self._dense(b)
            phase = torch.remainder(self.t - inj.epoch + 0.5 * P, P) - 0.5 * P
            tau = phase / dur + 0.5
            x = tau.clamp(0.0, 1.0) * (dense.shape[0] - 1)
            i0 = x.floor().clamp(max=dense.shape[0] - 2).long()
            w = x - i0
            shape = dense[i0] * (1.0 - w) + dense[i0 + 1] * w
            shape = torch.where((tau >= 0.0) & (tau <= 1.0), shape, torch.zeros_like(shape))
            off = off + depth * shape
            injs.append(inj)
        return self.t, off.to(torch.float32), self.sigma, injs


class LearnedCurves:
    """Light curves of the learned-proposal workload generated on a torch
    device, with the recipe of learned_curve (80 000 points at 2 min, Poisson
    (1.5) gaps of U(0.2, 2) d, per-point sigma log-normal around 800 ppm with
    log-sd 0.25, half the curves with one planet: P log-uniform 1-100 d,
    depth log-uniform 50-3000 ppm, b uniform 0-0.9 rounded to 0.01, the
    duration of a circular orbit around a Sun-density star).  Points inside
    gaps keep their times and get a NaN sigma, which the search treats as
    missing.  The noise comes from a seeded device generator, the gap and
    injection parameters from a seeded numpy generator.  draw() returns
    device (t, f, sigma) and the injections."""

    def __init__(self, seed: int, device="cuda", planet_frac: float = 0.5):
        import torch
        self.torch = torch
        self.device = device
        self.n = LEARNED_N_POINTS
        self.cadence = 120.0 / DAY_S
        self.t = torch.arange(self.n, dtype=torch.float64, device=device) * self.cadence
        self.span = float((self.n - 1) * self.cadence)
        self.rng = np.random.default_rng(seed)
        self.gen = torch.Generator(device=device)
        self.gen.manual_seed(int(seed))
        self.planet_frac = planet_frac
        self.dense = {}

    def _dense(self, b: float):
        if b not in self.dense:
            self.dense[b] = self.torch.as_tensor(transit.dense_template(b=b), device=self.device)
        return self.dense[b]

    def draw(self):
        torch = self.torch
        keep = torch.ones(self.n, dtype=torch.bool, device=self.device)
        for _ in range(self.rng.poisson(1.5)):
            glen = self.rng.uniform(0.2, 2.0)
            g0 = self.rng.uniform(0.0, max(self.span - glen, 1e-9))
            keep &= ~((self.t >= g0) & (self.t < g0 + glen))
        sig = 800e-6 * torch.exp(0.25 * torch.randn(self.n, generator=self.gen, dtype=torch.float64,
                                                       device=self.device))
        off = -sig * torch.randn(self.n, generator=self.gen, dtype=torch.float64, device=self.device)
        injs = []
        if self.rng.uniform() < self.planet_frac:
            P = float(np.exp(self.rng.uniform(np.log(LEARNED_P_RANGE[0]), np.log(LEARNED_P_RANGE[1]))))
            b = round(round(float(self.rng.uniform(0.0, 0.9)) / 0.01) * 0.01, 6)
            dur = transit.transit_duration_days(P, b)
            depth = float(np.exp(self.rng.uniform(np.log(50e-6), np.log(3000e-6))))
            inj = Injection(P, float(self.rng.uniform(0.0, P)), dur, depth, b)
            dense = self._dense(b)
            phase = torch.remainder(self.t - inj.epoch + 0.5 * P, P) - 0.5 * P
            tau = phase / dur + 0.5
            x = tau.clamp(0.0, 1.0) * (dense.shape[0] - 1)
            i0 = x.floor().clamp(max=dense.shape[0] - 2).long()
            w = x - i0
            shape = dense[i0] * (1.0 - w) + dense[i0 + 1] * w
            shape = torch.where((tau >= 0.0) & (tau <= 1.0), shape, torch.zeros_like(shape))
            off = off + depth * shape
            injs.append(inj)
        sigma = torch.where(keep, sig, torch.full_like(sig, float("nan"))).to(torch.float32)
        return self.t, off.to(torch.float32), sigma, injs
