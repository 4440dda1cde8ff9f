"""ctypes declarations of the C ABI in include/cbct.h (marshalling only)."""

from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbct.so")

CBCT_OK = 0
CBCT_EINVAL = -1
CBCT_ENOMEM = -2
CBCT_EHIP = -3
CBCT_ENONFINITE = -4

KERNELS = ("pad", "project", "cells", "gather", "tv_sweep", "tv_energy", "other", "eq2")


class cbct_geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("au", ctypes.c_double), ("av", ctypes.c_double),
                ("sad", ctypes.c_double), ("sdd", ctypes.c_double),
                ("n_views", ctypes.c_int32), ("angles", ctypes.POINTER(ctypes.c_double)),
                ("step", ctypes.c_double), ("u_off", ctypes.c_double), ("v_off", ctypes.c_double),
                ("x_off", ctypes.c_double), ("y_off", ctypes.c_double), ("z_off", ctypes.c_double)]


MAX_LEVELS = 4  # CBCT_MAX_LEVELS


class cbct_fbs_params(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("n_levels", ctypes.c_int32),
                ("iters", ctypes.c_int32 * MAX_LEVELS), ("beta", ctypes.c_double * MAX_LEVELS),
                ("eps", ctypes.c_double), ("n_inner", ctypes.c_int32 * MAX_LEVELS),
                ("trace_energy", ctypes.c_int32), ("gradient", ctypes.c_int32),
                ("tol", ctypes.c_double)]


class cbct_fbs_report(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("E_eps", ctypes.c_double),
                ("E1", ctypes.c_double), ("E2", ctypes.c_double),
                ("beta_used", ctypes.c_double * MAX_LEVELS),
                ("n_inner_used", ctypes.c_int32 * MAX_LEVELS),
                ("level_iters", ctypes.c_int32 * MAX_LEVELS), ("iters_done", ctypes.c_int32),
                ("change", ctypes.c_double * MAX_LEVELS),
                ("trace", ctypes.POINTER(ctypes.c_double))]


# name -> (restype, argtypes); every symbol declared in include/cbct.h
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_D = ctypes.c_double
SIGNATURES = {
    "cbct_plan_create": (ctypes.c_int, [ctypes.POINTER(cbct_geom), ctypes.POINTER(_P)]),
    "cbct_plan_destroy": (None, [_P]),
    "cbct_plan_samples": (ctypes.c_int64, [_P]),
    "cbct_plan_geom": (ctypes.c_int, [_P, ctypes.POINTER(cbct_geom)]),
    "cbct_project": (ctypes.c_int, [_P, _P, _P, _P]),
    "cbct_project_residual": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "cbct_backproject": (ctypes.c_int, [_P, _P, _P, _P]),
    "cbct_backproject_update": (ctypes.c_int, [_P, _P, _P, _D, _P, _P]),
    "cbct_project_f64": (ctypes.c_int, [_P, _P, _P, _P]),
    "cbct_backproject_f64": (ctypes.c_int, [_P, _P, _P, _P]),
    "cbct_tv_prox": (ctypes.c_int, [ctypes.POINTER(cbct_geom), _P, _P, _D, _D, _I32, _D, _I32, _P]),
    "cbct_tv_prox_noalloc": (ctypes.c_int, [ctypes.POINTER(cbct_geom), _P, _P, _D, _D, _I32,
                                            _D, _I32, _P]),
    "cbct_tv_energy": (ctypes.c_int, [ctypes.POINTER(cbct_geom), _P, _D,
                                      ctypes.POINTER(_D), _P]),
    "cbct_plan_lambda": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_D), _P]),
    "cbct_fbs_solve": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(cbct_fbs_params),
                                      ctypes.POINTER(cbct_fbs_report), _P]),
    "cbct_fbs_init": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(cbct_fbs_params),
                                     ctypes.POINTER(_P), _P]),
    "cbct_fbs_step": (ctypes.c_int, [_P, _I32, _P]),
    "cbct_fbs_finished": (ctypes.c_int, [_P]),
    "cbct_fbs_report_get": (ctypes.c_int, [_P, ctypes.POINTER(cbct_fbs_report)]),
    "cbct_fbs_free": (None, [_P]),
    "cbct_fbs_footprint": (ctypes.c_size_t, [ctypes.POINTER(cbct_geom),
                                             ctypes.POINTER(cbct_fbs_params)]),
    "cbct_kernel_timing": (ctypes.c_int, [_I32]),
    "cbct_kernel_timing_select": (ctypes.c_int, [ctypes.c_uint32]),
    "cbct_kernel_timing_read": (ctypes.c_int, [_I32, ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(_D)]),
    "cbct_probe_fma_rate": (ctypes.c_int, [_I32, ctypes.POINTER(_D), _P]),
    "cbct_backproject_eq2": (ctypes.c_int, [_P, _P, _P, _P]),
    "cbct_log_counts": (ctypes.c_int, [_P, _P, _D, _D, _P, ctypes.c_int64, _P]),
    "cbct_kernel_config": (ctypes.c_int, [ctypes.POINTER(_I32), _I32]),
    "cbct_projector_tile_margin": (ctypes.c_int, [ctypes.POINTER(cbct_geom), ctypes.POINTER(_I32)]),
    "cbct_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "cbct_last_error": (ctypes.c_char_p, []),
}

_lock = threading.Lock()
_lib = None


class CbctError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        super().__init__("%s failed (%d): %s" % (where, code, detail))


def lib():
    """The loaded libcbct.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libcbct.so is not built; run "
                                  "`python -m paper_1002_3675_amd.build` (needs hipcc)")
            h = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(h, name)
                fn.restype = res
                fn.argtypes = args
            _lib = h
    return _lib


def check(rc, where):
    if rc != CBCT_OK:
        detail = lib().cbct_last_error().decode(errors="replace")
        raise CbctError(rc, where, detail)
    return rc
