"""Quadratic limb-darkened transit shapes, used as *input data*.

The search method takes a densely sampled transit template as an input (the
paper ships such templates, generated with a third-party package, for
R_p = 0.03 R_*, b in {0.32, 0.93, 0.99} and quadratic limb darkening
u1, u2 = 0.4804, 0.1867; Sec. 2.1.2).  That package is not available here,
so this module computes the same kind of shape from textbook geometry:

* stellar intensity I(r) = 1 - u1 (1 - mu) - u2 (1 - mu)^2, mu = sqrt(1 - r^2);
* total stellar flux  F = pi (1 - u1/3 - u2/6);
* blocked flux of a dark disc of radius p at projected separation z,
  written as an integral over stellar radius r of I(r) times the length of the
  arc of the circle of radius r that lies inside the planet disc.

The planet crosses the stellar disc on a straight chord at impact parameter b
(the large-orbit limit), so in time normalised from first (tau = 0) to last
(tau = 1) contact the shape depends only on (p, b, u1, u2).

This module holds no step of the search itself: it only manufactures inputs
(the dense template and injected signals).
"""

from __future__ import annotations

import functools

import numpy as np

DEFAULT_P = 0.03
DEFAULT_B = 0.32
DEFAULT_U1 = 0.4804
DEFAULT_U2 = 0.1867

_GL_NODES = 96


@functools.lru_cache(maxsize=None)
def _gauss_legendre(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    # map [-1, 1] -> [0, 1]
    return 0.5 * (x + 1.0), 0.5 * w


def intensity(r, u1: float, u2: float):
    """Quadratic limb-darkening law, normalised to 1 at disc centre."""
    r = np.asarray(r, dtype=np.float64)
    mu = np.sqrt(np.clip(1.0 - r * r, 0.0, None))
    one_mu = 1.0 - mu
    return 1.0 - u1 * one_mu - u2 * one_mu * one_mu


def stellar_flux(u1: float, u2: float) -> float:
    """Integral of ``intensity`` over the unit disc (closed form)."""
    return np.pi * (1.0 - u1 / 3.0 - u2 / 6.0)


def _arc_angle(r, z: float, p: float):
    """Half-angle of the circle of radius r (about the star centre) that lies
    inside the planet disc of radius p centred at distance z."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    inside = r <= p - z  # whole circle inside the planet disc (only if z < p)
    out[inside] = np.pi
    part = (~inside) & (r > abs(z - p)) & (r < z + p)
    if np.any(part):
        rr = r[part]
        c = (rr * rr + z * z - p * p) / (2.0 * rr * z)
        out[part] = np.arccos(np.clip(c, -1.0, 1.0))
    return out


def _integrate_piece(a: float, b: float, fn) -> float:
    """Integral of fn over [a, b] with a cosine change of variable that
    removes square-root endpoint behaviour, then Gauss-Legendre."""
    if b <= a:
        return 0.0
    s, w = _gauss_legendre(_GL_NODES)
    half = 0.5 * (b - a)
    r = a + half * (1.0 - np.cos(np.pi * s))
    dr = half * np.pi * np.sin(np.pi * s)
    return float(np.sum(w * fn(r) * dr))


def blocked_fraction(z: float, p: float = DEFAULT_P, u1: float = DEFAULT_U1,
                     u2: float = DEFAULT_U2) -> float:
    """Fraction of the stellar flux hidden by the planet at separation z."""
    z = float(abs(z))
    if z >= 1.0 + p:
        return 0.0

    def integrand(r):
        return intensity(r, u1, u2) * 2.0 * r * _arc_angle(r, z, p)

    total = 0.0
    r_hi = min(1.0, z + p)
    if z < p:
        # full circles out to p - z, then partial arcs
        k = min(p - z, 1.0)
        total += _integrate_piece(0.0, k, lambda r: intensity(r, u1, u2) * 2.0 * np.pi * r)
        total += _integrate_piece(k, r_hi, integrand)
    else:
        r_lo = z - p
        # the stellar limb (r = 1) and the arc ends are the only non-smooth
        # points; both are interval ends here
        total += _integrate_piece(r_lo, r_hi, integrand)
    return total / stellar_flux(u1, u2)


def overlap_area(z: float, p: float) -> float:
    """Area of the intersection of the unit disc and a disc of radius p at
    centre distance z (two-circle lens area; textbook geometry)."""
    z = float(abs(z))
    if z >= 1.0 + p:
        return 0.0
    if z <= 1.0 - p:
        return np.pi * p * p
    if z <= p - 1.0:
        return np.pi
    k0 = np.arccos((p * p + z * z - 1.0) / (2.0 * p * z))
    k1 = np.arccos((1.0 - p * p + z * z) / (2.0 * z))
    s = 4.0 * z * z - (1.0 + z * z - p * p) ** 2
    return p * p * k0 + k1 - 0.5 * np.sqrt(max(s, 0.0))


def chord_separation(tau, p: float, b: float):
    """Projected separation along a straight chord at impact parameter b, with
    tau = 0 at first contact and tau = 1 at last contact."""
    tau = np.asarray(tau, dtype=np.float64)
    xc = np.sqrt((1.0 + p) ** 2 - b * b)
    x = xc * (2.0 * tau - 1.0)
    return np.sqrt(x * x + b * b)


@functools.lru_cache(maxsize=128)
def _dense_shape_cached(n: int, p: float, b: float, u1: float, u2: float):
    tau = np.linspace(0.0, 1.0, n)
    z = chord_separation(tau, p, b)
    d = np.array([blocked_fraction(zz, p, u1, u2) for zz in z])
    peak = d.max()
    if peak <= 0.0:
        raise ValueError("transit does not occult the star (b >= 1 + p)")
    d = d / peak
    d.setflags(write=False)
    return d


def dense_template(n: int = 4097, p: float = DEFAULT_P, b: float = DEFAULT_B,
                   u1: float = DEFAULT_U1, u2: float = DEFAULT_U2) -> np.ndarray:
    """Densely sampled transit shape over contact-normalised time, FP64,
    normalised to a maximum offset of 1 (first sample = first contact, last
    sample = last contact).  This is the form of template the search takes."""
    if b >= 1.0 + p:
        raise ValueError("impact parameter too large for a transit")
    return _dense_shape_cached(int(n), float(p), float(b), float(u1), float(u2)).copy()


def shape_at(tau, dense: np.ndarray):
    """Evaluate a dense template at contact-normalised times tau (zero outside
    [0, 1]) by linear interpolation.  Used to inject signals."""
    tau = np.asarray(tau, dtype=np.float64)
    x = np.linspace(0.0, 1.0, dense.shape[0])
    out = np.interp(tau, x, dense, left=0.0, right=0.0)
    out[(tau < 0.0) | (tau > 1.0)] = 0.0
    return out


def transit_duration_days(period: float, b: float, p: float = DEFAULT_P,
                          rho_star_solar: float = 1.0) -> float:
    """First-to-last-contact duration (days) of a circular orbit around a star
    of the given mean density (solar units), from Kepler's third law:
    a/R_* = (G rho_* P^2 / (3 pi))^(1/3), T14 = P/pi * asin(sqrt((1+p)^2-b^2) / (a/R_*))
    (small-angle-free, circular orbit, i from b = a cos i / R_*)."""
    G = 6.674e-11
    rho_sun = 1408.0  # kg m^-3
    P = period * 86400.0
    a_over_r = (G * rho_star_solar * rho_sun * P * P / (3.0 * np.pi)) ** (1.0 / 3.0)
    if b >= a_over_r:
        return 0.0
    sin_i = np.sqrt(1.0 - (b / a_over_r) ** 2)
    arg = np.sqrt(max((1.0 + p) ** 2 - b * b, 0.0)) / (a_over_r * sin_i)
    arg = min(arg, 1.0)
    return period / np.pi * np.arcsin(arg)
