"""ctypes declarations mirroring include/nssdoa.h, and the loader of libnssdoa.so.

The library is required: importing the binding without a built library raises, so no caller can
silently fall back to anything else.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnssdoa.so")

# enums
OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, ESTATE = range(6)
ALGS = {"phd": 0, "music": 1, "ev": 2, "mn": 3}
PRECS = {"c128": 0, "c64": 1, "bf16": 2, "f16": 3}
WS_COV, WS_EVALS, WS_EVECS, WS_B, WS_QREF, WS_SPECTRUM = range(6)
STAGES = {"covariance": 0, "eigen": 1, "scan": 2, "peaks": 3, "proposal": 4}
ST_NONFINITE_INPUT = 0x1
ST_EVD_NOT_CONVERGED = 0x2
ST_DEGENERATE = 0x4
ST_FEWER_PEAKS = 0x8
ST_PEAK_OVERFLOW = 0x10
ST_FALLBACK_USED = 0x20


class Array(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pos_wl", ctypes.POINTER(ctypes.c_double))]


class Grid(ctypes.Structure):
    _fields_ = [("start_deg", ctypes.c_double), ("step_deg", ctypes.c_double),
                ("L", ctypes.c_int32), ("circular", ctypes.c_int32),
                ("polar_start_deg", ctypes.c_double), ("polar_step_deg", ctypes.c_double),
                ("n_polar", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [("array_id", ctypes.c_int32), ("grid_id", ctypes.c_int32),
                ("N", ctypes.c_int32), ("D", ctypes.c_int32),
                ("x_off", ctypes.c_int64), ("ldx", ctypes.c_int64), ("spec_off", ctypes.c_int64)]


class Peak(ctypes.Structure):
    _fields_ = [("idx", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("angle_deg", ctypes.c_double), ("value", ctypes.c_double), ("polar_deg", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("eig_tol", ctypes.c_double), ("eig_max_iter", ctypes.c_int32),
                ("refine_halfwidth", ctypes.c_int32), ("lowq_tau", ctypes.c_double),
                ("extra_candidates", ctypes.c_int32), ("scan_rows", ctypes.c_int32),
                ("eig_method", ctypes.c_int32), ("c64_scan", ctypes.c_int32)]


EIG_METHODS = {"auto": 0, "ql": 1, "jacobi": 2}
C64_SCANS = {"split3": 0, "fp32": 1, "split16": 2}
SCAN_FORMS = {"factored": 0, "quadratic": 1, "complement": 2}


PEAK_DTYPE = np.dtype([("idx", "<i4"), ("reserved", "<i4"), ("angle_deg", "<f8"), ("value", "<f8"),
                       ("polar_deg", "<f8")])
assert PEAK_DTYPE.itemsize == ctypes.sizeof(Peak) == 32
assert ctypes.sizeof(Grid) == 48

_P = ctypes.c_void_p
_SIGNATURES = {
    "nssdoa_plan_create": [ctypes.POINTER(_P), ctypes.POINTER(Array), ctypes.c_int32,
                           ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(Options)],
    "nssdoa_plan_destroy": [_P],
    "nssdoa_batch_create": [ctypes.POINTER(_P), _P, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(Frame), ctypes.c_int32, ctypes.c_int32],
    "nssdoa_batch_destroy": [_P],
    "nssdoa_workspace_size": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "nssdoa_workspace_offset": [_P, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "nssdoa_estimate": [_P, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P, _P, _P, _P,
                        ctypes.c_size_t, _P],
    "nssdoa_estimate_noalloc": [_P, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P, _P, _P, _P],
    "nssdoa_noalloc_workspace_limit": [ctypes.POINTER(ctypes.c_size_t)],
    "nssdoa_set_timing": [_P, ctypes.c_int32],
    "nssdoa_stage_time": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_int64)],
    "nssdoa_mlp_create": [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "nssdoa_mlp_destroy": [_P],
    "nssdoa_mlp_param_count": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "nssdoa_mlp_save": [_P, _P, ctypes.POINTER(ctypes.c_size_t)],
    "nssdoa_mlp_load": [_P, _P, ctypes.c_size_t],
    "nssdoa_mlp_forward": [_P, _P, ctypes.c_int32, _P, _P],
    "nssdoa_mlp_train_step": [_P, _P, _P, ctypes.c_int32, ctypes.c_float, _P, _P],
    "nssdoa_mlp_gradients": [_P, _P, ctypes.c_size_t],
    "nssdoa_windowed_workspace_size": [_P, _P, ctypes.POINTER(ctypes.c_size_t)],
    "nssdoa_features": [_P, _P, ctypes.c_size_t, _P, ctypes.c_int32, _P],
    "nssdoa_scan_form": [_P, ctypes.c_int32, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P],
    "nssdoa_graph_create": [ctypes.POINTER(_P), _P, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P, _P, _P, _P,
                            ctypes.c_size_t],
    "nssdoa_graph_launch": [_P, _P],
    "nssdoa_pipeline_create": [ctypes.POINTER(_P), _P, ctypes.c_int32],
    "nssdoa_pipeline_submit": [_P, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)],
    "nssdoa_pipeline_wait": [_P, ctypes.c_int64],
    "nssdoa_pipeline_destroy": [_P],
    "nssdoa_graph_destroy": [_P],
    "nssdoa_estimate_windowed": [_P, _P, ctypes.c_size_t, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_float, ctypes.c_float, ctypes.c_int32, _P, ctypes.c_size_t, _P, _P, _P,
                                 _P, ctypes.c_size_t, _P],
    "nssdoa_estimate_learned": [_P, _P, _P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int32, _P, ctypes.c_size_t, _P, _P, _P, _P,
                                ctypes.c_size_t, _P],
}

_lib = None


def load(path: str = None) -> ctypes.CDLL:
    """Load libnssdoa.so (once) and declare its prototypes; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libnssdoa.so is not built (%s); run __graft_entry__.build() first" % path)
    lib = ctypes.CDLL(path)
    for name, args in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.nssdoa_status_string.argtypes = [ctypes.c_int]
    lib.nssdoa_status_string.restype = ctypes.c_char_p
    lib.nssdoa_last_error.argtypes = []
    lib.nssdoa_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class NssdoaError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        super().__init__("%s failed with status %d: %s" % (func, status, message))
        self.status = status


def check(status: int, func: str) -> None:
    if status != OK:
        msg = load().nssdoa_last_error().decode(errors="replace")
        raise NssdoaError(status, func, msg)
