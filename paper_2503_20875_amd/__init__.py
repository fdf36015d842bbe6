"""MI355X transit search: Python binding of ``libcetra.so``.

Thin wrappers with the C ABI's names (``include/cetra.h``): they allocate
output tensors with PyTorch (device memory only), pass raw pointers and the
current HIP stream, and check the returned status.  All arithmetic runs in
the library's HIP kernels; importing the package does not load the library,
but the first call does and fails loudly if it has not been built.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _abi
from ._abi import BestRecord, CetraError, Grid, Tuning  # noqa: F401

__all__ = ["BatchPlan", "batch_plan", "batch_search", "get_tuning", "set_tuning", "reset_tuning", "grid_plan", "template_resample", "resample", "linear_search", "loglike0",
           "periodic_workspace", "periodic_search", "best", "search", "Grid", "CetraError"]


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dev(x, dtype):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        if x.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {x.dtype}")
        return x.contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def version() -> int:
    return int(_abi.load().cetra_version())


def get_tuning() -> dict:
    t = Tuning()
    _abi.check(_abi.load().cetra_get_tuning(ctypes.byref(t)))
    return dict(fold_period_block=t.fold_period_block, fold_wgs_per_cu=t.fold_wgs_per_cu,
                fold_units_per_wg=t.fold_units_per_wg, fold_variant=t.fold_variant,
                linear_windows=t.linear_windows)


def set_tuning(fold_period_block: int = 8, fold_wgs_per_cu: int = 8, fold_units_per_wg: int = 4,
               fold_variant: int = 2, linear_windows: int = 4) -> None:
    t = Tuning(fold_period_block, fold_wgs_per_cu, fold_units_per_wg, fold_variant, linear_windows)
    _abi.check(_abi.load().cetra_set_tuning(ctypes.byref(t)))


def reset_tuning() -> None:
    _abi.check(_abi.load().cetra_set_tuning(None))


def grid_plan(t_first: float, t_last: float, cadence: float, durations, t0_step: float = 0.0,
              n_model: int = 1024) -> Grid:
    durs = np.ascontiguousarray(durations, dtype=np.float64)
    g = Grid()
    _abi.check(_abi.load().cetra_grid_plan(float(t_first), float(t_last), float(cadence),
                                           durs.ctypes.data_as(ctypes.c_void_p), int(durs.shape[0]),
                                           float(t0_step), int(n_model), ctypes.byref(g)))
    return g


SOLAR_DENSITY = 1.408  # g cm^-3


def period_grid(span: float, p_min: float, p_max: float, rho: float = SOLAR_DENSITY,
                oversample: float = 3.0) -> np.ndarray:
    """Optimally sampled period grid (ascending, days): evenly spaced in
    f^(1/3), one step moving the last transit of the span by 1/oversample of
    a central transit's duty cycle around a star of density rho (g/cm^3)."""
    lib = _abi.load()
    n = ctypes.c_int64()
    _abi.check(lib.cetra_period_grid(float(span), float(p_min), float(p_max), float(rho), float(oversample),
                                     None, 0, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.float64)
    _abi.check(lib.cetra_period_grid(float(span), float(p_min), float(p_max), float(rho), float(oversample),
                                     out.ctypes.data_as(ctypes.c_void_p), out.shape[0], ctypes.byref(n)))
    return out


def duration_limits(period: float, rho_min: float, rho_max: float, k_max: float = 0.2,
                    b_max: float = 0.9) -> tuple:
    """(d_min, d_max) in days: the Keplerian transit-duration range of one
    period for circular orbits around stars of density [rho_min, rho_max]."""
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _abi.check(_abi.load().cetra_duration_limits(float(period), float(rho_min), float(rho_max), float(k_max),
                                                 float(b_max), ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


def keplerian_jrange(periods, durations, rho_min: float, rho_max: float, k_max: float = 0.2,
                     b_max: float = 0.9) -> np.ndarray:
    """int32 [K][2] duration-index ranges (host) for periodic_search's jrange:
    the durations inside each period's Keplerian limits."""
    p = np.ascontiguousarray(periods, dtype=np.float64)
    d = np.ascontiguousarray(durations, dtype=np.float64)
    out = np.empty((p.shape[0], 2), dtype=np.int32)
    _abi.check(_abi.load().cetra_keplerian_jrange(p.ctypes.data_as(ctypes.c_void_p), p.shape[0],
                                                  d.ctypes.data_as(ctypes.c_void_p), d.shape[0], float(rho_min),
                                                  float(rho_max), float(k_max), float(b_max),
                                                  out.ctypes.data_as(ctypes.c_void_p)))
    return out


def template_resample(dense, n_model: int = 1024, stream=None):
    torch = _torch()
    d = _dev(dense, torch.float64)
    out = torch.empty(n_model, dtype=torch.float32, device=d.device)
    _abi.check(_abi.load().cetra_template_resample(_stream(stream), _ptr(d), d.numel(), int(n_model), _ptr(out)))
    return out


def resample(grid: Grid, t, f, sigma, status: bool = True, stream=None):
    """Returns (flux, ivar, status_tensor_or_None)."""
    torch = _torch()
    t = _dev(t, torch.float64)
    f = _dev(f, torch.float32)
    s = _dev(sigma, torch.float32)
    if not (t.numel() == f.numel() == s.numel()):
        raise ValueError("t, f, sigma must have the same length")
    flux = torch.empty(grid.n, dtype=torch.float32, device=t.device)
    ivar = torch.empty(grid.n, dtype=torch.float32, device=t.device)
    st = torch.empty(1, dtype=torch.int32, device=t.device) if status else None
    _abi.check(_abi.load().cetra_resample(_stream(stream), ctypes.byref(grid), _ptr(t), _ptr(f), _ptr(s),
                                          t.numel(), _ptr(flux), _ptr(ivar), _ptr(st)))
    return flux, ivar, st


def linear_search(grid: Grid, flux, ivar, model, public: bool = False, fold=None, stream=None):
    """Returns fold [J, I, 2] (and depth, var, lr [J, I] if public)."""
    torch = _torch()
    shape = (grid.n_dur, grid.n_t0)
    dev = flux.device
    if fold is None:
        fold = torch.empty(shape + (2,), dtype=torch.float32, device=dev)
    depth = var = lr = None
    if public:
        depth = torch.empty(shape, dtype=torch.float32, device=dev)
        var = torch.empty(shape, dtype=torch.float32, device=dev)
        lr = torch.empty(shape, dtype=torch.float32, device=dev)
    _abi.check(_abi.load().cetra_linear_search(_stream(stream), ctypes.byref(grid), _ptr(flux), _ptr(ivar),
                                               _ptr(model), _ptr(fold), _ptr(depth), _ptr(var), _ptr(lr)))
    if public:
        return fold, depth, var, lr
    return fold


def loglike0(grid: Grid, flux, ivar, stream=None):
    torch = _torch()
    out = torch.empty(1, dtype=torch.float64, device=flux.device)
    _abi.check(_abi.load().cetra_loglike0(_stream(stream), ctypes.byref(grid), _ptr(flux), _ptr(ivar),
                                          _ptr(out)))
    return out


def periodic_workspace(grid: Grid, n_eval: int) -> int:
    n = ctypes.c_size_t()
    _abi.check(_abi.load().cetra_periodic_workspace(ctypes.byref(grid), int(n_eval), ctypes.byref(n)))
    return int(n.value)


def epoch_strides(grid: Grid, fraction: float = 0.01) -> np.ndarray:
    """int32 [J] (host) epoch strides for periodic_search's `stride`: per
    duration, the largest whole number of reference-time steps not above
    `fraction` of the duration (a step that grows with the duration)."""
    out = np.empty(grid.n_dur, dtype=np.int32)
    _abi.check(_abi.load().cetra_epoch_strides(ctypes.byref(grid), float(fraction),
                                               out.ctypes.data_as(ctypes.c_void_p)))
    return out


def periodic_search(grid: Grid, fold, periods, jrange=None, subset=None, work=None, out=None,
                    stream=None, stride=None) -> dict:
    """Per-period maximum-likelihood records: dict of device tensors
    lr, epoch, dur, depth, depth_var ([K] each).  `stride` (host ints, one
    per duration, >= 1) evaluates only the epochs that are multiples of it."""
    torch = _torch()
    dev = fold.device
    periods = _dev(periods, torch.float64)
    K = periods.numel()
    jr = None if jrange is None else _dev(jrange, torch.int32)
    sub = None if subset is None else _dev(subset, torch.int64)
    n_eval = K if sub is None else sub.numel()
    need = periodic_workspace(grid, n_eval)
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if out is None:
        out = dict(lr=torch.empty(K, dtype=torch.float32, device=dev),
                   epoch=torch.empty(K, dtype=torch.int32, device=dev),
                   dur=torch.empty(K, dtype=torch.int32, device=dev),
                   depth=torch.empty(K, dtype=torch.float32, device=dev),
                   depth_var=torch.empty(K, dtype=torch.float32, device=dev))
    if stride is None:
        _abi.check(_abi.load().cetra_periodic_search(
            _stream(stream), ctypes.byref(grid), _ptr(fold), _ptr(periods), K, _ptr(jr), _ptr(sub),
            0 if sub is None else sub.numel(), _ptr(work), work.numel(), _ptr(out["lr"]), _ptr(out["epoch"]),
            _ptr(out["dur"]), _ptr(out["depth"]), _ptr(out["depth_var"])))
        return out
    st = np.ascontiguousarray(stride, dtype=np.int32)
    if st.shape != (grid.n_dur,):
        raise ValueError(f"stride: one value per duration ({grid.n_dur})")
    _abi.check(_abi.load().cetra_periodic_search_strided(
        _stream(stream), ctypes.byref(grid), _ptr(fold), _ptr(periods), K, _ptr(jr), _ptr(sub),
        0 if sub is None else sub.numel(), st.ctypes.data_as(ctypes.c_void_p), _ptr(work), work.numel(),
        _ptr(out["lr"]), _ptr(out["epoch"]), _ptr(out["dur"]), _ptr(out["depth"]), _ptr(out["depth_var"])))
    return out


def periodic_search_noalloc(grid: Grid, fold, periods, jrange=None, subset=None, out=None,
                            stream=None) -> dict:
    """periodic_search with the library's fixed device scratch as the fold
    workspace (the C call allocates nothing; `out` may be passed in so this
    wrapper allocates nothing either).  Calls that overlap on one device
    share the scratch and race."""
    torch = _torch()
    dev = fold.device
    periods = _dev(periods, torch.float64)
    K = periods.numel()
    jr = None if jrange is None else _dev(jrange, torch.int32)
    sub = None if subset is None else _dev(subset, torch.int64)
    if out is None:
        out = dict(lr=torch.empty(K, dtype=torch.float32, device=dev),
                   epoch=torch.empty(K, dtype=torch.int32, device=dev),
                   dur=torch.empty(K, dtype=torch.int32, device=dev),
                   depth=torch.empty(K, dtype=torch.float32, device=dev),
                   depth_var=torch.empty(K, dtype=torch.float32, device=dev))
    _abi.check(_abi.load().cetra_periodic_search_noalloc(
        _stream(stream), ctypes.byref(grid), _ptr(fold), _ptr(periods), K, _ptr(jr), _ptr(sub),
        0 if sub is None else sub.numel(), _ptr(out["lr"]), _ptr(out["epoch"]), _ptr(out["dur"]),
        _ptr(out["depth"]), _ptr(out["depth_var"])))
    return out


def periodic_search_noalloc_limit(grid: Grid) -> int:
    """Most evaluated periods periodic_search_noalloc accepts."""
    n = ctypes.c_int64()
    _abi.check(_abi.load().cetra_periodic_search_noalloc_limit(ctypes.byref(grid), ctypes.byref(n)))
    return int(n.value)


def best(grid: Grid, periods, per: dict, out=None, stream=None):
    """Best period; returns a uint8 device tensor holding one cetra_best_record
    (use ``best_record`` to read it on the host)."""
    torch = _torch()
    periods = _dev(periods, torch.float64)
    if out is None:
        out = torch.empty(ctypes.sizeof(BestRecord), dtype=torch.uint8, device=periods.device)
    _abi.check(_abi.load().cetra_best(_stream(stream), ctypes.byref(grid), _ptr(periods), periods.numel(),
                                      _ptr(per["lr"]), _ptr(per["epoch"]), _ptr(per["dur"]), _ptr(per["depth"]),
                                      _ptr(per["depth_var"]), _ptr(out)))
    return out


def single_events(grid: Grid, fold, n_events: int = 5, out=None, stream=None):
    """The n strongest non-overlapping single-transit candidates of a
    linear search (fold-ready [J][I][2]); returns a uint8 device tensor of
    n cetra_event records (``event_records`` reads them on the host)."""
    torch = _torch()
    n = int(n_events)
    if not 1 <= n <= _abi.MAX_EVENTS:
        raise ValueError(f"n_events must lie in [1, {_abi.MAX_EVENTS}]")
    size = ctypes.c_size_t()
    _abi.check(_abi.load().cetra_single_events_workspace(n, ctypes.byref(size)))
    work = torch.empty(size.value, dtype=torch.uint8, device=fold.device)
    if out is None:
        out = torch.empty((n, ctypes.sizeof(_abi.Event)), dtype=torch.uint8, device=fold.device)
    _abi.check(_abi.load().cetra_single_events(_stream(stream), ctypes.byref(grid), _ptr(fold), n, _ptr(work),
                                               work.numel(), _ptr(out)))
    return out


def event_records(raw) -> list:
    """Host copies of the cetra_event records written by ``single_events``."""
    data = raw.cpu().numpy()
    recs = []
    for row in data.reshape(-1, ctypes.sizeof(_abi.Event)):
        e = _abi.Event.from_buffer_copy(bytes(row.tobytes()))
        recs.append({name: getattr(e, name) for name, _ in _abi.Event._fields_})
    return recs


def mask_transits(grid: Grid, flux, ivar, period: float, t0: float, duration: float, width: float = 1.5,
                  stream=None) -> None:
    """Null (in place) the resampled points within width * duration / 2 of
    every transit t0 + n P (t0 relative to the grid origin); a period that is
    not finite and positive masks the single event at t0."""
    _abi.check(_abi.load().cetra_mask_transits(_stream(stream), ctypes.byref(grid), float(period), float(t0),
                                               float(duration), float(width), _ptr(flux), _ptr(ivar)))


def iterative_search(t, f, sigma, cadence: float, durations, periods, dense, n_signals: int = 3,
                     mask_width: float = 1.5, n_model: int = 1024, t0_step: float = 0.0, jrange=None,
                     stream=None) -> list:
    """Multi-signal search: after each search the strongest periodic signal
    is nulled in the resampled light curve (mask_transits) and the linear
    and periodic searches run again.  Returns the best record of every
    pass (a pass that finds nothing ends the loop)."""
    torch = _torch()
    t_host = np.asarray(t) if not hasattr(t, "cpu") else t.cpu().numpy()
    grid = grid_plan(t_host[0], t_host[-1], cadence, durations, t0_step, n_model)
    model = template_resample(dense, n_model, stream=stream)
    flux, ivar, _ = resample(grid, t, f, sigma, status=False, stream=stream)
    per_d = _dev(periods, torch.float64)
    K = per_d.numel()
    work = torch.empty(max(periodic_workspace(grid, K), 1), dtype=torch.uint8, device=per_d.device)
    fold = per = None
    found = []
    for _ in range(int(n_signals)):
        fold = linear_search(grid, flux, ivar, model, fold=fold, stream=stream)
        per = periodic_search(grid, fold, per_d, jrange=jrange, work=work, out=per, stream=stream)
        b = best_record(best(grid, per_d, per, stream=stream))
        found.append(b)
        if b["k"] < 0:
            break
        mask_transits(grid, flux, ivar, b["period"], b["t0"], b["duration"], mask_width, stream=stream)
    return found


def multi_template_search(t, f, sigma, cadence: float, durations, periods, denses, n_model: int = 1024,
                          t0_step: float = 0.0, jrange=None, stream=None) -> dict:
    """The search run once per template (e.g. a sequence of impact
    parameters, Sec. 2.1.2) on one resampled light curve, merged per period
    (cetra_periodic_merge: largest LR, ties to the earlier template).
    Returns the merged per-period records, the winning template per period
    ("set") and the best record with its template index."""
    torch = _torch()
    t_host = np.asarray(t) if not hasattr(t, "cpu") else t.cpu().numpy()
    grid = grid_plan(t_host[0], t_host[-1], cadence, durations, t0_step, n_model)
    flux, ivar, _ = resample(grid, t, f, sigma, status=False, stream=stream)
    per_d = _dev(periods, torch.float64)
    K = per_d.numel()
    T = len(denses)
    dev = per_d.device
    stack = dict(lr=torch.empty((T, K), dtype=torch.float32, device=dev),
                 epoch=torch.empty((T, K), dtype=torch.int32, device=dev),
                 dur=torch.empty((T, K), dtype=torch.int32, device=dev),
                 depth=torch.empty((T, K), dtype=torch.float32, device=dev),
                 depth_var=torch.empty((T, K), dtype=torch.float32, device=dev))
    work = torch.empty(max(periodic_workspace(grid, K), 1), dtype=torch.uint8, device=dev)
    fold = None
    for s_, dense in enumerate(denses):
        model = template_resample(dense, n_model, stream=stream)
        fold = linear_search(grid, flux, ivar, model, fold=fold, stream=stream)
        periodic_search(grid, fold, per_d, jrange=jrange, work=work, out={k: v[s_] for k, v in stack.items()},
                        stream=stream)
    out = {k: torch.empty(K, dtype=v.dtype, device=dev) for k, v in stack.items()}
    out["set"] = torch.empty(K, dtype=torch.int32, device=dev)
    _abi.check(_abi.load().cetra_periodic_merge(_stream(stream), T, K, _ptr(stack["lr"]), _ptr(stack["epoch"]),
                                                _ptr(stack["dur"]), _ptr(stack["depth"]), _ptr(stack["depth_var"]),
                                                _ptr(out["lr"]), _ptr(out["epoch"]), _ptr(out["dur"]),
                                                _ptr(out["depth"]), _ptr(out["depth_var"]), _ptr(out["set"])))
    per = {k: out[k] for k in ("lr", "epoch", "dur", "depth", "depth_var")}
    b = best_record(best(grid, per_d, per, stream=stream))
    b["template"] = int(out["set"][b["k"]].item()) if b["k"] >= 0 else -1
    return dict(grid=grid, periodic=per, set=out["set"], best=b)


def best_record(raw) -> dict:
    """Host copy of a cetra_best_record produced by ``best``."""
    b = BestRecord.from_buffer_copy(bytes(raw.cpu().numpy().tobytes()))
    return {name: getattr(b, name) for name, _ in BestRecord._fields_}


def search(t, f, sigma, cadence: float, durations, periods, dense, n_model: int = 1024,
           t0_step: float = 0.0, public: bool = False, jrange=None, subset=None, stream=None) -> dict:
    """Whole path on the current device: template resampling, light-curve
    resampling, linear search, periodic search, best period."""
    t_host = np.asarray(t) if not hasattr(t, "cpu") else t.cpu().numpy()
    grid = grid_plan(t_host[0], t_host[-1], cadence, durations, t0_step, n_model)
    model = template_resample(dense, n_model, stream=stream)
    flux, ivar, st = resample(grid, t, f, sigma, stream=stream)
    lin = linear_search(grid, flux, ivar, model, public=public, stream=stream)
    fold = lin[0] if public else lin
    per = periodic_search(grid, fold, periods, jrange=jrange, subset=subset, stream=stream)
    b = best(grid, periods, per, stream=stream)
    out = dict(grid=grid, model=model, flux=flux, ivar=ivar, fold=fold, periodic=per, best_raw=b, status=st)
    if public:
        out.update(depth=lin[1], var=lin[2], lr=lin[3])
    return out


# ------------------------------------------------------------------- batches
class BatchPlan:
    """Host-side plan of a batch (owns the C plan object)."""

    def __init__(self, handle, info, n_curves: int, period_offsets):
        self._h = handle
        self.info = {name: getattr(info, name) for name, _ in _abi.BatchInfo._fields_}
        self.n_curves = n_curves
        self.period_offsets = np.asarray(period_offsets, dtype=np.int64)
        self._cancel = None

    @property
    def handle(self):
        return self._h

    def order(self) -> np.ndarray:
        o = np.zeros(self.n_curves, dtype=np.int32)
        _abi.check(_abi.load().cetra_batch_plan_order(self._h, o.ctypes.data_as(ctypes.c_void_p), self.n_curves))
        return o

    def tables(self) -> bytes:
        """The plan's tables image (copied to the start of a workspace)."""
        buf = ctypes.create_string_buffer(max(self.info["tables_bytes"], 1))
        _abi.check(_abi.load().cetra_batch_tables(self._h, buf, len(buf)))
        return buf.raw[: self.info["tables_bytes"]]

    def cancel_flag(self):
        """The plan's pinned-host cancel flag (a ctypes int32 pointer):
        setting ``flag[0] = 1`` while a search runs stops it early."""
        if self._cancel is None:
            p = ctypes.POINTER(ctypes.c_int32)()
            _abi.check(_abi.load().cetra_batch_cancel_flag(self._h, ctypes.byref(p)))
            self._cancel = p
        return self._cancel

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            try:
                _abi.load().cetra_batch_plan_destroy(h)
            except Exception:
                pass


def batch_plan(grids, obs_offsets, period_offsets, period_block: int = 0, shuffle_seed: int = 0,
               pop_items: int = 0) -> BatchPlan:
    """Plan a batch from per-curve grid plans and CSR offsets (host arrays).
    pop_items: work items a workgroup takes per queue pop (0: chosen at
    launch)."""
    n = len(grids)
    garr = (Grid * n)(*grids)
    oo = np.ascontiguousarray(obs_offsets, dtype=np.int64)
    po = np.ascontiguousarray(period_offsets, dtype=np.int64)
    if oo.shape[0] != n + 1 or po.shape[0] != n + 1:
        raise ValueError("offsets must have n_curves + 1 entries")
    d = _abi.BatchDesc(n, int(period_block), ctypes.cast(garr, ctypes.c_void_p), oo.ctypes.data_as(ctypes.c_void_p),
                       po.ctypes.data_as(ctypes.c_void_p), int(shuffle_seed), int(pop_items), 0)
    lib = _abi.load()
    h = ctypes.c_void_p()
    _abi.check(lib.cetra_batch_plan_create(ctypes.byref(d), ctypes.byref(h)))
    info = _abi.BatchInfo()
    _abi.check(lib.cetra_batch_plan_info(h, ctypes.byref(info)))
    return BatchPlan(h, info, n, po)


def batch_workspace(plan: BatchPlan, device="cuda"):
    """Device workspace of the plan's size with the plan's tables copied to
    its start (one host-to-device copy; searches only read them)."""
    torch = _torch()
    work = torch.empty(max(plan.info["workspace_bytes"], 1), dtype=torch.uint8, device=device)
    tbl = torch.frombuffer(bytearray(plan.tables()), dtype=torch.uint8)
    work[: tbl.numel()].copy_(tbl)
    return work


def batch_search(plan: BatchPlan, t, f, sigma, model, periods, work=None, out=None, cancel=None,
                 resume: bool = False, jrange=None, stream=None) -> dict:
    """Search every curve of the batch with one persistent launch.  Returns
    device tensors: per-period lr, epoch, dur, depth, depth_var (CSR), best
    records (uint8 [n_curves, sizeof(cetra_best_record)]), done [n_curves]
    and status.  `cancel`: None (the plan's flag, if made), or an int32
    device tensor; `resume` skips curves whose done flag is set in `out`;
    `jrange` (int32 [total periods, 2], CSR like the periods) restricts each
    period's durations."""
    torch = _torch()
    jr = None if jrange is None else _dev(jrange, torch.int32)
    t = _dev(t, torch.float64)
    f = _dev(f, torch.float32)
    s = _dev(sigma, torch.float32)
    periods = _dev(periods, torch.float64)
    dev = t.device
    if work is None:
        work = batch_workspace(plan, dev)
    K = int(plan.period_offsets[-1])
    if out is None:
        out = dict(lr=torch.empty(max(K, 1), dtype=torch.float32, device=dev),
                   epoch=torch.empty(max(K, 1), dtype=torch.int32, device=dev),
                   dur=torch.empty(max(K, 1), dtype=torch.int32, device=dev),
                   depth=torch.empty(max(K, 1), dtype=torch.float32, device=dev),
                   depth_var=torch.empty(max(K, 1), dtype=torch.float32, device=dev),
                   best=torch.empty((plan.n_curves, ctypes.sizeof(BestRecord)), dtype=torch.uint8, device=dev),
                   done=torch.zeros(plan.n_curves, dtype=torch.int32, device=dev),
                   status=torch.empty(1, dtype=torch.int32, device=dev))
    _abi.check(_abi.load().cetra_batch_search(
        plan.handle, _stream(stream), _ptr(t), _ptr(f), _ptr(s), _ptr(model), _ptr(periods), _ptr(jr), _ptr(cancel),
        _abi.BATCH_RESUME if resume else 0, _ptr(work), work.numel(), _ptr(out["lr"]), _ptr(out["epoch"]),
        _ptr(out["dur"]), _ptr(out["depth"]), _ptr(out["depth_var"]), _ptr(out["best"]), _ptr(out["done"]),
        _ptr(out["status"])))
    return out


def best_records(raw) -> list:
    """Host copies of a [n, sizeof(cetra_best_record)] device tensor."""
    data = raw.cpu().numpy()
    return [best_record_bytes(bytes(row.tobytes())) for row in data]


def best_record_bytes(b: bytes) -> dict:
    r = BestRecord.from_buffer_copy(b)
    return {name: getattr(r, name) for name, _ in BestRecord._fields_}
