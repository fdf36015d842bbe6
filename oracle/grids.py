"""Oracle for the default period and duration grids (Sec. 2.1.3) -- TEST
INFRASTRUCTURE ONLY.

Plain FP64 numpy written from the definitions: the paper adopts TLS's grids,
that is the optimally sampled period grid of Ofir (2014) and, per period,
only the transit durations a Keplerian orbit allows.  Only the tests may
import this module; it shares no code with the GPU package.

* Circular orbit around a star of mean density rho: Kepler's third law with
  M = 4/3 pi R^3 rho gives (a/R)^3 = G rho P^2 / (3 pi).
* First-to-last-contact duration with radius ratio k and impact parameter b:
  T = (P/pi) asin(sqrt((1+k)^2 - b^2) / ((a/R) sin i)), cos i = b / (a/R).
* Duty cycle of a central transit of a small planet: q = T/P ~ (R/a)/pi,
  which is (3 pi / (G rho))^(1/3) f^(2/3) / pi in terms of frequency f.
* Optimal sampling: consecutive frequencies differ by the step that moves
  the last transit of the span S by q / oversample of a phase, df = q / (S os).
  Since q grows as f^(2/3), that step is constant in f^(1/3).
"""

from __future__ import annotations

import numpy as np

G_CGS = 6.67430e-8   # cm^3 g^-1 s^-2
DAY_S = 86400.0


def a_over_r(period_days, rho):
    """Orbital semi-major axis in stellar radii (Kepler's third law)."""
    p = np.asarray(period_days, dtype=np.float64) * DAY_S
    return np.cbrt(G_CGS * rho * p * p / (3.0 * np.pi))


def t14(period_days, rho, k, b):
    """First-to-last-contact duration (days) of a circular orbit; half the
    period when the orbit lies inside the star, 0 when it does not transit."""
    P = float(period_days)
    ar = float(a_over_r(P, rho))
    chord2 = (1.0 + k) ** 2 - b * b
    if chord2 <= 0.0 or b / ar >= 1.0:
        return 0.0
    sin_i = np.sqrt(1.0 - (b / ar) ** 2)
    x = np.sqrt(chord2) / (ar * sin_i)
    if x >= 1.0:
        return 0.5 * P
    return P / np.pi * np.arcsin(x)


def duration_limits(period_days, rho_min, rho_max, k_max, b_max):
    """(d_min, d_max): a grazing-limited transit (b = b_max, k = 0) across the
    densest star and a central transit of the largest planet (k = k_max,
    b = 0) across the least dense star."""
    return t14(period_days, rho_max, 0.0, b_max), t14(period_days, rho_min, k_max, 0.0)


def duty_cycle(freq_per_s, rho):
    """Duty cycle (R/a)/pi of a central transit at frequency f (s^-1)."""
    return np.cbrt(3.0 * np.pi / (G_CGS * rho)) * np.power(freq_per_s, 2.0 / 3.0) / np.pi


def period_grid(span_days, p_min, p_max, rho, oversample):
    """Ascending periods (days): frequencies from 1/p_max upward in equal
    steps of f^(1/3), (3 pi / (G rho))^(1/3) / (3 pi S os), for as long as
    the period stays >= p_min."""
    S = span_days * DAY_S
    step = np.cbrt(3.0 * np.pi / (G_CGS * rho)) / (3.0 * np.pi * S * oversample)
    x0 = np.cbrt(1.0 / (p_max * DAY_S))
    x1 = np.cbrt(1.0 / (p_min * DAY_S))
    n = int(np.floor((x1 - x0) / step)) + 1
    x = x0 + step * np.arange(n, dtype=np.float64)
    return (1.0 / x ** 3 / DAY_S)[::-1].copy()


def keplerian_jrange(periods, durations, rho_min, rho_max, k_max, b_max):
    """int32 [K][2]: first and last duration index inside each period's
    limits (lo > hi when none), by a plain scan of every (period, duration)."""
    durations = np.asarray(durations, dtype=np.float64)
    out = np.empty((len(periods), 2), dtype=np.int32)
    for k, P in enumerate(periods):
        lo_d, hi_d = duration_limits(P, rho_min, rho_max, k_max, b_max)
        inside = [j for j, D in enumerate(durations) if lo_d <= D <= hi_d]
        first = next((j for j, D in enumerate(durations) if D >= lo_d), len(durations))
        last = max((j for j, D in enumerate(durations) if D <= hi_d), default=-1)
        assert not inside or (inside[0] == first and inside[-1] == last)
        out[k] = (first, last)
    return out


def epoch_strides(durations, t0_step, fraction):
    """int32 [J]: per duration, the fold's epoch stride on the fixed
    reference-time grid for a TLS-style step that grows with the duration
    (Sec. 2.1.3 mentions adopting it): the largest multiple of the fixed step
    not exceeding `fraction` of the duration, and at least one step.  The
    1e-9 keeps exact ratios (D_j a whole multiple of D_min) from landing one
    short by rounding."""
    out = np.empty(len(durations), dtype=np.int32)
    for j, D in enumerate(durations):
        q = fraction * float(D) / t0_step
        out[j] = max(1, int(np.floor(q + 1e-9)))
    return out
