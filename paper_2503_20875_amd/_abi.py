"""ctypes declarations of the C ABI in ``include/cetra.h``.

Argument marshalling only: every computation happens in ``libcetra.so``.
Loading fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcetra.so")
MAX_DURATIONS = 64
MAX_MODEL = 4096

STATUS = {0: "CETRA_OK", -1: "CETRA_ERR_INVALID", -2: "CETRA_ERR_RANGE", -3: "CETRA_ERR_WORKSPACE",
          -4: "CETRA_ERR_HIP", -5: "CETRA_ERR_DEVICE"}


class CetraError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Grid(ctypes.Structure):
    """Mirror of ``cetra_grid``."""
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
        ("durations", ctypes.c_double * MAX_DURATIONS),
        ("dur_step_fx", ctypes.c_uint64 * MAX_DURATIONS),
    ]


class Event(ctypes.Structure):
    """Mirror of ``cetra_event``."""
    _fields_ = [
        ("epoch", ctypes.c_int32),
        ("dur", ctypes.c_int32),
        ("t0", ctypes.c_double),
        ("t0_abs", ctypes.c_double),
        ("duration", ctypes.c_double),
        ("lr", ctypes.c_double),
        ("depth", ctypes.c_double),
        ("depth_var", ctypes.c_double),
        ("snr", ctypes.c_double),
    ]


MAX_EVENTS = 64


class BestRecord(ctypes.Structure):
    """Mirror of ``cetra_best_record``."""
    _fields_ = [
        ("k", ctypes.c_int64),
        ("epoch", ctypes.c_int32),
        ("dur", ctypes.c_int32),
        ("period", ctypes.c_double),
        ("duration", ctypes.c_double),
        ("t0", ctypes.c_double),
        ("t0_abs", ctypes.c_double),
        ("lr", ctypes.c_double),
        ("depth", ctypes.c_double),
        ("depth_var", ctypes.c_double),
        ("snr", ctypes.c_double),
    ]


class Tuning(ctypes.Structure):
    """Mirror of ``cetra_tuning``."""
    _fields_ = [
        ("fold_period_block", ctypes.c_int32),
        ("fold_wgs_per_cu", ctypes.c_int32),
        ("fold_units_per_wg", ctypes.c_int32),
        ("fold_variant", ctypes.c_int32),
        ("linear_windows", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class BatchDesc(ctypes.Structure):
    """Mirror of ``cetra_batch_desc``."""
    _fields_ = [
        ("n_curves", ctypes.c_int32),
        ("fold_period_block", ctypes.c_int32),
        ("grids", ctypes.c_void_p),
        ("obs_offsets", ctypes.c_void_p),
        ("period_offsets", ctypes.c_void_p),
        ("shuffle_seed", ctypes.c_int64),
        ("pop_items", ctypes.c_int32),
        ("reserved1", ctypes.c_int32),
    ]


class BatchInfo(ctypes.Structure):
    """Mirror of ``cetra_batch_info``."""
    _fields_ = [
        ("workspace_bytes", ctypes.c_size_t),
        ("tables_bytes", ctypes.c_size_t),
        ("n_curves", ctypes.c_int64),
        ("total_periods", ctypes.c_int64),
        ("n_launches", ctypes.c_int64),
        ("n_items", ctypes.c_int64),
        ("n_slots", ctypes.c_int32),
        ("period_block", ctypes.c_int32),
        ("lds_bytes", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class ShapeClass(ctypes.Structure):
    """Mirror of ``cetra_shape_class``."""
    _fields_ = [
        ("arch", ctypes.c_char * 32),
        ("log2_t0", ctypes.c_int32),
        ("n_dur", ctypes.c_int32),
        ("log2_periods", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


BATCH_RESUME = 1
BATCH_CANCELLED, BATCH_WAIT_LIMIT, BATCH_BAD_TABLES, BATCH_UNSORTED = 1, 2, 4, 8


_P = ctypes.c_void_p
_i32, _i64, _d, _sz, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_float

# name -> (restype, argtypes); the list is the ABI's export list
SIGNATURES = {
    "cetra_version": (ctypes.c_int, []),
    "cetra_last_error": (ctypes.c_char_p, []),
    "cetra_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "cetra_get_tuning": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
    "cetra_set_tuning": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
    "cetra_grid_plan": (ctypes.c_int, [_d, _d, _d, _P, _i32, _d, _i32, ctypes.POINTER(Grid)]),
    "cetra_period_grid": (ctypes.c_int, [_d, _d, _d, _d, _d, _P, _i64, _P]),
    "cetra_single_events_workspace": (ctypes.c_int, [_i32, ctypes.POINTER(ctypes.c_size_t)]),
    "cetra_single_events": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _P, _i32, _P, ctypes.c_size_t, _P]),
    "cetra_mask_transits": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _d, _d, _d, _d, _P, _P]),
    "cetra_periodic_merge": (ctypes.c_int, [_P, _i32, _i64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "cetra_duration_limits": (ctypes.c_int, [_d, _d, _d, _d, _d, _P, _P]),
    "cetra_keplerian_jrange": (ctypes.c_int, [_P, _i64, _P, _i32, _d, _d, _d, _d, _P]),
    "cetra_template_resample": (ctypes.c_int, [_P, _P, _i64, _i32, _P]),
    "cetra_resample": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _P, _P, _P, _i64, _P, _P, _P]),
    "cetra_linear_search": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _P, _P]),
    "cetra_loglike0": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _P, _P, _P]),
    "cetra_periodic_workspace": (ctypes.c_int, [ctypes.POINTER(Grid), _i64, ctypes.POINTER(_sz)]),
    "cetra_periodic_search": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _P, _P, _i64, _P, _P, _i64, _P, _sz,
                                             _P, _P, _P, _P, _P]),
    "cetra_periodic_search_strided": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _P, _P, _i64, _P, _P, _i64, _P,
                                                     _P, _sz, _P, _P, _P, _P, _P]),
    "cetra_epoch_strides": (ctypes.c_int, [ctypes.POINTER(Grid), _d, _P]),
    "cetra_periodic_search_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _P, _P, _i64, _P, _P, _i64, _P, _P,
                                                     _P, _P, _P]),
    "cetra_periodic_search_noalloc_limit": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(_i64)]),
    "cetra_best": (ctypes.c_int, [_P, ctypes.POINTER(Grid), _P, _i64, _P, _P, _P, _P, _P, _P]),
    "cetra_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(BatchDesc), ctypes.POINTER(_P)]),
    "cetra_batch_plan_destroy": (ctypes.c_int, [_P]),
    "cetra_batch_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(BatchInfo)]),
    "cetra_batch_plan_order": (ctypes.c_int, [_P, _P, _i32]),
    "cetra_shape_class_of": (ctypes.c_int, [ctypes.POINTER(Grid), _i64, ctypes.POINTER(ShapeClass)]),
    "cetra_autotune_workspace": (ctypes.c_int, [ctypes.POINTER(Grid), _i64, ctypes.POINTER(_sz)]),
    "cetra_autotune": (ctypes.c_int, [_P, ctypes.POINTER(ShapeClass), ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _i64,
                                      _P, _sz, ctypes.c_char_p, ctypes.POINTER(Tuning), ctypes.POINTER(_d),
                                      ctypes.POINTER(_d), ctypes.POINTER(_i32)]),
    "cetra_batch_workspace": (ctypes.c_int, [_P, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "cetra_batch_tables": (ctypes.c_int, [_P, _P, _sz]),
    "cetra_batch_cancel_flag": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))]),
    "cetra_batch_search": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _i32, _P, _sz, _P, _P, _P, _P, _P,
                                          _P, _P, _P]),
    "cetra_net_mfma_probe": (ctypes.c_int, [_P, _P, _P, _P]),
    "cetra_net_downsample": (ctypes.c_int, [_P, _P, _i32, _i64, _i32, _P]),
    "cetra_net_downsample_signed": (ctypes.c_int, [_P, _P, _i32, _i64, _i32, _P]),
    "cetra_conv1d_fwd": (ctypes.c_int, [_P, _P, _i32, _i32, _i32, _P, _i32, _P, _P]),
    "cetra_conv1d_bwd": (ctypes.c_int, [_P, _P, _P, _P, _i32, _i32, _i32, _P, _i32, _P, _P, _P, _i64, _P, _P, _P]),
    "cetra_conv1d_bwd_partial_floats": (ctypes.c_int64, [_i32, _i32, _i32]),
    "cetra_net_project_fwd": (ctypes.c_int, [_P, _P, _i64, _P, _P, _i32, _P]),
    "cetra_net_project_bwd": (ctypes.c_int, [_P, _P, _P, _i64, _P, _i32, _P, _P, _P]),
    "cetra_net_foldpool_fwd": (ctypes.c_int, [_P, _P, _i32, _i32, _i32, _P, _i32, _i32, _P, _P, _P]),
    "cetra_net_foldpool_bwd": (ctypes.c_int, [_P, _P, _P, _P, _i32, _i32, _i32, _i32, _i32, _P]),
    "cetra_net_head_fwd": (ctypes.c_int, [_P, _P, _i64, _i32, _P, _P, _P, _P, _i32, _P]),
    "cetra_net_bce": (ctypes.c_int, [_P, _P, _P, _i64, _f32, _P, _P]),
    "cetra_net_head_bwd": (ctypes.c_int, [_P, _P, _i64, _i32, _P, _P, _P, _i32, _P, _P, _P, _P, _P, _P]),
    "cetra_adam_step": (ctypes.c_int, [_P, _P, _P, _P, _P, _i64, _f32, _f32, _f32, _f32, _i64]),
    "cetra_net_pack_conv_w": (ctypes.c_int, [_P, _P, _i32, _i32, _P]),
    "cetra_topk_windows": (ctypes.c_int, [_P, _P, _i32, _i32, _i32, _P]),
    "cetra_windows_to_periods": (ctypes.c_int, [_P, _P, _i64, _P, _i32, _P, _i32, _P, _P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libcetra.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_2503_20875_amd.build.build() "
                          "(there is no CPU fallback for the GPU path)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != 0:
        msg = load().cetra_last_error()
        raise CetraError(status, msg.decode() if msg else "")
