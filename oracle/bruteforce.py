"""Brute-force transit search for tiny inputs -- TEST INFRASTRUCTURE ONLY.

Independent of ``oracle.c`` in every step:

* grid indices (resampling bin, window bounds, template sample, transit
  epoch) are computed in exact rational arithmetic (``fractions.Fraction``)
  from the FP64 inputs, not in FP64/fixed point;
* the transit model of a candidate is built as an explicit vector over *all*
  N resampled points (zero outside its windows);
* the depth is the exact least-squares solution of the full Gaussian
  log-likelihood (Eq. 1) over all N points, its variance the inverse Fisher
  information, and the likelihood ratio the difference of the full Eq. 1
  log-likelihoods (including the log-normalisation terms) between that model
  and the zero-offset model;
* the periodic search builds the summed multi-transit model vector and fits
  one common depth in the same way; its argmax is exhaustive.

The grid conventions follow the same readings as the oracle (window
[t_i - D/2, t_i + D/2], null if it leaves [0, (N-1)c]; nearest cell-centred
template sample; nearest reference time for each transit; a period shorter
than the reference-time step, or not finite, is not evaluated).
"""

from __future__ import annotations

import math
from fractions import Fraction as Fr

import numpy as np


class BruteGrid:
    def __init__(self, t_first, t_last, cadence, durations, n_model, t0_step=0.0):
        self.t_first = float(t_first)
        self.c = float(cadence)
        self.durations = [float(d) for d in durations]
        self.M = int(n_model)
        dmax, dmin = max(self.durations), min(self.durations)
        c = Fr(self.c)
        self.n_pad = math.ceil(Fr(dmax) / 2 / c)
        self.n_data = math.floor((Fr(float(t_last)) - Fr(self.t_first)) / c + Fr(1, 2)) + 1
        self.N = self.n_data + 2 * self.n_pad
        self.dt = float(t0_step) if t0_step > 0 else 0.01 * dmin
        self.I = math.floor((self.N - 1) * c / Fr(self.dt)) + 1

    def resample(self, t, f, sigma):
        """Inverse-variance mean per nearest grid point, in FP64 sums."""
        N = self.N
        w = np.zeros(N)
        fw = np.zeros(N)
        members = [[] for _ in range(N)]
        for n in range(len(t)):
            s = float(sigma[n])
            if not (np.isfinite(t[n]) and np.isfinite(f[n]) and np.isfinite(s) and s > 0):
                continue
            q = self.n_pad + math.floor((Fr(float(t[n])) - Fr(self.t_first)) / Fr(self.c) + Fr(1, 2))
            if 0 <= q < N:
                members[q].append(n)
        for q in range(N):
            if members[q]:
                ws = np.array([1.0 / float(sigma[n]) ** 2 for n in members[q]])
                fs = np.array([float(f[n]) for n in members[q]])
                w[q] = ws.sum()
                fw[q] = (ws * fs).sum()
        flux = np.where(w > 0, fw / np.where(w > 0, w, 1.0), 0.0)
        return flux, w

    def window_model(self, i, j, model):
        """Explicit model vector (length N) of the window (i, j), or None if null."""
        c, D = Fr(self.c), Fr(self.durations[j])
        ts = i * Fr(self.dt) - D / 2
        te = ts + D
        if ts < 0 or te > (self.N - 1) * c:
            return None
        lo = math.ceil(ts / c)
        hi = math.floor(te / c)
        if lo > hi:
            return None
        g = np.zeros(self.N)
        for n in range(lo, hi + 1):
            tau = (n * c - ts) / D
            k = min(self.M - 1, max(0, math.floor(tau * self.M)))
            g[n] = float(model[k])
        return g

    def evaluates(self, period):
        """Whether the periodic search evaluates this period at all."""
        return bool(np.isfinite(period)) and Fr(float(period)) >= Fr(self.dt)

    def transit_epochs(self, i, period):
        """Grid epochs i + round_half_up(m P / dt), m = 0, 1, ... inside the grid."""
        out = []
        m = 0
        step = Fr(float(period)) / Fr(self.dt)
        while True:
            x = i + math.floor(m * step + Fr(1, 2))
            if x >= self.I:
                return out
            out.append(x)
            m += 1

    def epochs_per_period(self, period):
        return min(self.I, math.ceil(Fr(float(period)) / Fr(self.dt)))


def loglike(g, depth, flux, w):
    """Gaussian log-likelihood (Eq. 1, normalisation included) of the model
    depth * g over every resampled point with finite uncertainty
    (sigma^2 = 1/w); null points (w = 0) carry no information."""
    ok = w > 0
    lnorm = -0.5 * np.log(2 * np.pi / w[ok])
    return float(np.sum(-0.5 * w[ok] * (depth * g[ok] - flux[ok]) ** 2 + lnorm))


def fit(g, flux, w):
    """Least-squares depth of model g on all points, its variance, and the
    full-Eq.-1 log-likelihood ratio against the zero-offset model."""
    ok = w > 0
    a = float(np.sum(w[ok] * g[ok] * flux[ok]))
    b = float(np.sum(w[ok] * g[ok] * g[ok]))
    if b <= 0:
        return None
    z = a / b
    return z, 1.0 / b, loglike(g, z, flux, w) - loglike(g, 0.0, flux, w)


def linear(bg: BruteGrid, flux, w, model, elements=None):
    """Brute-force linear search; elements: iterable of (j, i) or None = all."""
    if elements is None:
        elements = [(j, i) for j in range(len(bg.durations)) for i in range(bg.I)]
    out = {}
    for (j, i) in elements:
        g = bg.window_model(i, j, model)
        out[(j, i)] = None if g is None else fit(g, flux, w)
    return out


def periodic(bg: BruteGrid, flux, w, model, periods, windows=None, stride=None):
    """Exhaustive periodic search: per period, best (lr, i, j, z, zvar).
    Windows are cached per (i, j) across periods.  With `stride`, duration j
    tries only the epochs that are multiples of stride[j]."""
    cache = {} if windows is None else windows

    def win(i, j):
        if (i, j) not in cache:
            cache[(i, j)] = bg.window_model(i, j, model)
        return cache[(i, j)]

    results = []
    for P in periods:
        best = None
        if not bg.evaluates(P):
            results.append(best)
            continue
        for j, D in enumerate(bg.durations):
            if not D < P:
                continue
            for i in range(0, bg.epochs_per_period(P), 1 if stride is None else int(stride[j])):
                g = np.zeros(bg.N)
                any_win = False
                for x in bg.transit_epochs(i, P):
                    gx = win(x, j)
                    if gx is not None:
                        g += gx
                        any_win = True
                if not any_win:
                    continue
                r = fit(g, flux, w)
                if r is None:
                    continue
                if best is None or r[2] > best[0]:
                    best = (r[2], i, j, r[0], r[1])
        results.append(best)
    return results
