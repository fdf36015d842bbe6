"""Binding of the library's launch autotuner (``cetra_autotune``).

The timing loop, the candidate set and the JSON cache keyed by GPU
architecture and shape class live in the library; this module marshals the
arguments.  ``tune`` returns the tuning it applied (see
``cetra_set_tuning``) with the measured or cached times.
"""

from __future__ import annotations

import ctypes

from . import _abi, _dev, _ptr, _stream


def shape_class(grid, n_periods: int, arch: str = "") -> _abi.ShapeClass:
    sc = _abi.ShapeClass()
    _abi.check(_abi.load().cetra_shape_class_of(ctypes.byref(grid), int(n_periods), ctypes.byref(sc)))
    sc.arch = arch.encode()
    return sc


def workspace_bytes(grid, n_periods: int) -> int:
    n = ctypes.c_size_t()
    _abi.check(_abi.load().cetra_autotune_workspace(ctypes.byref(grid), int(n_periods), ctypes.byref(n)))
    return int(n.value)


def tune(grid, flux, ivar, model, fold, periods, cache_path=None, arch: str = "", stream=None) -> dict:
    """Apply the cached or measured fastest tuning for this search's shape
    class.  `fold` [J, I, 2] is overwritten by linear searches (same values)
    when candidates are timed.  Returns dict(tuning=..., fold_ms, linear_ms,
    from_cache)."""
    import torch
    periods = _dev(periods, torch.float64)
    K = int(periods.numel())
    sc = shape_class(grid, K, arch)
    work = None
    if flux is not None:
        work = torch.empty(max(workspace_bytes(grid, K), 1), dtype=torch.uint8, device=periods.device)
    t = _abi.Tuning()
    fms, lms, hit = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    _abi.check(_abi.load().cetra_autotune(
        _stream(stream) if flux is not None else None, ctypes.byref(sc), ctypes.byref(grid), _ptr(flux), _ptr(ivar),
        _ptr(model), _ptr(fold), _ptr(periods), K, _ptr(work), 0 if work is None else work.numel(),
        None if cache_path is None else str(cache_path).encode(), ctypes.byref(t), ctypes.byref(fms),
        ctypes.byref(lms), ctypes.byref(hit)))
    tuning = {name: getattr(t, name) for name, _ in _abi.Tuning._fields_ if name != "reserved"}
    return dict(tuning=tuning, fold_ms=fms.value, linear_ms=lms.value, from_cache=bool(hit.value))
