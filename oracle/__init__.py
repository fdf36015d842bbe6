"""FP64 CPU oracle for the transit search -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct definitions of what the GPU library computes
(resampling, template resampling, the linear search with the paper's two
passes, the periodic search with the paper's common-depth fold, the best
period), written in C (``oracle.c``) and driven from here with ctypes, plus a
numpy brute force (``bruteforce.py``) for tiny inputs.

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this package.  It imports nothing from the GPU package and the GPU
package imports nothing from it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_DUR = 64
_lock = threading.Lock()
_lib = None


class Grid(ctypes.Structure):
    _fields_ = [
        ("t_first", ctypes.c_double),
        ("cadence", ctypes.c_double),
        ("t_origin", ctypes.c_double),
        ("t0_step", ctypes.c_double),
        ("n_pad", ctypes.c_int64),
        ("n_data", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("n_t0", ctypes.c_int64),
        ("n_dur", ctypes.c_int32),
        ("n_model", ctypes.c_int32),
        ("durations", ctypes.c_double * MAX_DUR),
        ("dur_step_fx", ctypes.c_uint64 * MAX_DUR),
    ]

    @property
    def durations_array(self) -> np.ndarray:
        return np.array(self.durations[: self.n_dur], dtype=np.float64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.POINTER
            d, i64, i32, f32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
            L.ora_grid_plan.argtypes = [d, d, d, P(d), i32, d, i32, P(Grid)]
            L.ora_grid_plan.restype = ctypes.c_int
            L.ora_template.argtypes = [P(d), i64, i32, P(f32)]
            L.ora_template.restype = None
            L.ora_resample.argtypes = [P(Grid), P(d), P(f32), P(f32), i64, P(d), P(d)]
            L.ora_resample.restype = None
            L.ora_linear.argtypes = [P(Grid), P(d), P(d), P(f32), P(d), P(d), P(d), P(d)]
            L.ora_linear.restype = None
            L.ora_linear_at.argtypes = [P(Grid), P(d), P(d), P(f32), P(i64), i64, P(d), P(d), P(d), P(d)]
            L.ora_linear_at.restype = None
            L.ora_loglike0.argtypes = [P(Grid), P(d), P(d)]
            L.ora_loglike0.restype = d
            L.ora_periodic.argtypes = [P(Grid), P(d), P(d), P(d), P(d), P(d), P(i32), P(i64), i64, P(i32),
                                       P(d), P(i32), P(i32), P(d), P(d), P(d)]
            L.ora_periodic.restype = None
            L.ora_fold_at.argtypes = [P(Grid), P(d), P(d), P(d), P(d), d, i64, i32, P(d), P(d), P(d), P(d)]
            L.ora_fold_at.restype = ctypes.c_int
            L.ora_best.argtypes = [P(d), P(i32), i64]
            L.ora_best.restype = i64
            L.ora_set_threads.argtypes = [ctypes.c_int]
            L.ora_max_threads.restype = ctypes.c_int
            _lib = L
    return _lib


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def max_threads() -> int:
    return int(lib().ora_max_threads())


def grid_plan(t_first: float, t_last: float, cadence: float, durations, n_model: int = 1024,
              t0_step: float = 0.0) -> Grid:
    durs = np.ascontiguousarray(durations, dtype=np.float64)
    g = Grid()
    rc = lib().ora_grid_plan(float(t_first), float(t_last), float(cadence), _p(durs, ctypes.c_double),
                             int(durs.shape[0]), float(t0_step), int(n_model), ctypes.byref(g))
    if rc != 0:
        raise ValueError("invalid grid parameters")
    return g


def template(dense, n_model: int = 1024) -> np.ndarray:
    dense = np.ascontiguousarray(dense, dtype=np.float64)
    out = np.empty(n_model, dtype=np.float32)
    lib().ora_template(_p(dense, ctypes.c_double), dense.shape[0], int(n_model), _p(out, ctypes.c_float))
    return out


def resample(g: Grid, t, f, sigma):
    t = np.ascontiguousarray(t, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float32)
    s = np.ascontiguousarray(sigma, dtype=np.float32)
    flux = np.empty(g.n, dtype=np.float64)
    ivar = np.empty(g.n, dtype=np.float64)
    lib().ora_resample(ctypes.byref(g), _p(t, ctypes.c_double), _p(f, ctypes.c_float),
                       _p(s, ctypes.c_float), t.shape[0], _p(flux, ctypes.c_double),
                       _p(ivar, ctypes.c_double))
    return flux, ivar


def linear(g: Grid, flux, ivar, model):
    """Full linear search; returns dict of [J, I] FP64 arrays."""
    flux = np.ascontiguousarray(flux, dtype=np.float64)
    ivar = np.ascontiguousarray(ivar, dtype=np.float64)
    model = np.ascontiguousarray(model, dtype=np.float32)
    shape = (g.n_dur, g.n_t0)
    out = {k: np.empty(shape, dtype=np.float64) for k in ("depth", "var", "lr", "aabs")}
    lib().ora_linear(ctypes.byref(g), _p(flux, ctypes.c_double), _p(ivar, ctypes.c_double),
                     _p(model, ctypes.c_float), *[_p(out[k], ctypes.c_double)
                                                  for k in ("depth", "var", "lr", "aabs")])
    return out


def linear_at(g: Grid, flux, ivar, model, idx):
    """Linear search at flat indices idx = j*I + i only."""
    flux = np.ascontiguousarray(flux, dtype=np.float64)
    ivar = np.ascontiguousarray(ivar, dtype=np.float64)
    model = np.ascontiguousarray(model, dtype=np.float32)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = {k: np.empty(idx.shape[0], dtype=np.float64) for k in ("depth", "var", "lr", "aabs")}
    lib().ora_linear_at(ctypes.byref(g), _p(flux, ctypes.c_double), _p(ivar, ctypes.c_double),
                        _p(model, ctypes.c_float), _p(idx, ctypes.c_int64), idx.shape[0],
                        *[_p(out[k], ctypes.c_double) for k in ("depth", "var", "lr", "aabs")])
    return out


def loglike0(g: Grid, flux, ivar) -> float:
    flux = np.ascontiguousarray(flux, dtype=np.float64)
    ivar = np.ascontiguousarray(ivar, dtype=np.float64)
    return float(lib().ora_loglike0(ctypes.byref(g), _p(flux, ctypes.c_double), _p(ivar, ctypes.c_double)))


def periodic(g: Grid, lin: dict, periods, jrange=None, sel=None, stride=None) -> dict:
    """Periodic search over periods[sel] (all periods if sel is None).  With
    `stride` ([J] int, >= 1), duration j evaluates only the epochs that are
    multiples of stride[j]."""
    periods = np.ascontiguousarray(periods, dtype=np.float64)
    if sel is None:
        sel = np.arange(periods.shape[0], dtype=np.int64)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    n = sel.shape[0]
    jr = None if jrange is None else np.ascontiguousarray(jrange, dtype=np.int32).reshape(-1)
    st = None if stride is None else np.ascontiguousarray(stride, dtype=np.int32)
    if st is not None and (st.shape != (g.n_dur,) or np.any(st < 1)):
        raise ValueError("stride: one integer >= 1 per duration")
    out = dict(lr=np.empty(n), i=np.empty(n, dtype=np.int32), j=np.empty(n, dtype=np.int32),
               z=np.empty(n), zvar=np.empty(n), aabs=np.empty(n))
    arrs = [np.ascontiguousarray(lin[k], dtype=np.float64) for k in ("depth", "var", "lr", "aabs")]
    lib().ora_periodic(ctypes.byref(g), *[_p(a, ctypes.c_double) for a in arrs],
                       _p(periods, ctypes.c_double),
                       None if jr is None else _p(jr, ctypes.c_int32),
                       _p(sel, ctypes.c_int64), n, None if st is None else _p(st, ctypes.c_int32),
                       _p(out["lr"], ctypes.c_double), _p(out["i"], ctypes.c_int32),
                       _p(out["j"], ctypes.c_int32), _p(out["z"], ctypes.c_double),
                       _p(out["zvar"], ctypes.c_double), _p(out["aabs"], ctypes.c_double))
    return out


def fold_at(g: Grid, lin: dict, period: float, i: int, j: int):
    """(lr, z, zvar, aabs) of one periodic candidate, or None if null."""
    arrs = [np.ascontiguousarray(lin[k], dtype=np.float64) for k in ("depth", "var", "lr", "aabs")]
    vals = [ctypes.c_double() for _ in range(4)]
    ok = lib().ora_fold_at(ctypes.byref(g), *[_p(a, ctypes.c_double) for a in arrs], float(period),
                           int(i), int(j), *[ctypes.byref(v) for v in vals])
    if not ok:
        return None
    return tuple(v.value for v in vals)


def best(per: dict) -> int:
    lr = np.ascontiguousarray(per["lr"], dtype=np.float64)
    i = np.ascontiguousarray(per["i"], dtype=np.int32)
    return int(lib().ora_best(_p(lr, ctypes.c_double), _p(i, ctypes.c_int32), lr.shape[0]))


def search(wl, t0_step: float = 0.0, jrange=None, sel=None, with_linear: bool = True) -> dict:
    """End-to-end oracle run on a workload (resample -> template -> linear ->
    periodic -> best)."""
    g = grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model, t0_step)
    model = template(wl.dense, wl.n_model)
    flux, ivar = resample(g, wl.t, wl.f, wl.sigma)
    lin = linear(g, flux, ivar, model)
    per = periodic(g, lin, wl.periods, jrange=jrange, sel=sel)
    kb = best(per)
    out = dict(grid=g, model=model, flux=flux, ivar=ivar, periodic=per, best=kb,
               loglike0=loglike0(g, flux, ivar))
    if with_linear:
        out["linear"] = lin
    return out
