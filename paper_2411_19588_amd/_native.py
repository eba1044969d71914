"""ctypes binding of libgsplash (include/gsplash.h): structures and prototypes only.

The product path has no fallback: if the HIP library is missing this module
raises on first use.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsplash.so")

GS_OK = 0
GS_ERR_INVALID_ARGUMENT = -1
GS_ERR_UNSUPPORTED = -2
GS_ERR_WORKSPACE_TOO_SMALL = -3
GS_ERR_HIP = -4
GS_STATUS_PAIR_OVERFLOW = 1
GS_STATUS_NONFINITE_INPUT = 2
GS_STATUS_INCOMPLETE = 4
GS_STATUS_TRUNCATED = GS_STATUS_PAIR_OVERFLOW | GS_STATUS_INCOMPLETE
GS_MAX_VIEWS = 64
GS_MAX_PAIRS = 2_147_483_647
GS_MAX_PHASES = 8
GS_FETCH_DEFAULT = 0
GS_FETCH_LDS = 1
GS_FETCH_SCALAR = 2
GS_STATE_STEP = 0
GS_STATE_SKIP = 1

_ERRORS = {GS_ERR_INVALID_ARGUMENT: "invalid argument", GS_ERR_UNSUPPORTED: "unsupported",
           GS_ERR_WORKSPACE_TOO_SMALL: "workspace too small", GS_ERR_HIP: "HIP runtime error"}


class GsError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {_ERRORS.get(code, code)} ({code})")
        self.code = code


class GsCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("near_z", ctypes.c_float)]


class GsGaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class GsGaussianGrads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class GsOptions(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("lds_batch", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("pixels_per_lane", ctypes.c_int32),
                ("record_fetch", ctypes.c_int32), ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("t_min", ctypes.c_float), ("dilation", ctypes.c_float), ("kappa", ctypes.c_float),
                ("depth_mode", ctypes.c_int32), ("tile_cull", ctypes.c_int32),
                ("phases", ctypes.c_int32), ("phase0_shift", ctypes.c_int32), ("depth_output", ctypes.c_int32),
                ("phase_growth", ctypes.c_int32), ("max_pairs", ctypes.c_int64), ("timer", ctypes.c_void_p),
                ("medium_prior", ctypes.c_void_p), ("prior_lambda", ctypes.c_float), ("reg_opacity", ctypes.c_float),
                ("reg_scale", ctypes.c_float), ("phase_limit", ctypes.c_int32)]


class GsAdamGroup(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("activated", ctypes.c_void_p), ("count", ctypes.c_int64),
                ("lr", ctypes.c_float), ("activation", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GsBackscatterOptions(ctypes.Structure):
    _fields_ = [("p_dark", ctypes.c_float), ("edges", ctypes.c_int32), ("intervals", ctypes.c_int32),
                ("resize_height", ctypes.c_int32)]


class GsMcmcState(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("param", ctypes.c_void_p * 5), ("m", ctypes.c_void_p * 5), ("v", ctypes.c_void_p * 5),
                ("scales", ctypes.c_void_p), ("opacity", ctypes.c_void_p)]


# Every symbol declared in include/gsplash.h, with (restype, argtypes).
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t
PROTOTYPES = {
    "gs_default_options": (None, [ctypes.POINTER(GsOptions)]),
    "gs_version": (ctypes.c_char_p, []),
    "gs_workspace_query": (ctypes.c_int, [ctypes.POINTER(GsOptions), _I64, _I32, ctypes.POINTER(GsCamera),
                                          ctypes.POINTER(_SZ), ctypes.POINTER(_SZ)]),
    "gs_render_forward": (ctypes.c_int, [ctypes.POINTER(GsOptions), ctypes.POINTER(GsGaussians), _I32,
                                         ctypes.POINTER(GsCamera), _P, _P, _P, _P, _P, _P, _P, _SZ, _P, _SZ, _P]),
    "gs_render_backward": (ctypes.c_int, [ctypes.POINTER(GsOptions), ctypes.POINTER(GsGaussians), _I32,
                                          ctypes.POINTER(GsCamera), _P, _P, _P, _P, _P, _P, _SZ,
                                          ctypes.POINTER(GsGaussianGrads), _P, _P, _SZ, _P]),
    "gs_render_backward_adam": (ctypes.c_int, [ctypes.POINTER(GsOptions), ctypes.POINTER(GsGaussians), _I32,
                                               ctypes.POINTER(GsCamera), _P, _P, _P, _P, _P, _P, _SZ,
                                               ctypes.POINTER(GsAdamGroup), ctypes.c_float, ctypes.c_float,
                                               ctypes.c_float, _P, _P, _SZ, _P]),
    "gs_read_status": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_I64), _P]),
    "gs_phases_needed": (ctypes.c_int, [ctypes.POINTER(GsOptions), _I64, _I32, ctypes.POINTER(GsCamera), _P, _SZ,
                                        ctypes.POINTER(_I32), _P]),
    "gs_export_keys": (ctypes.c_int, [ctypes.POINTER(GsOptions), _I64, _I32, ctypes.POINTER(GsCamera), _P, _SZ,
                                      _P, _P, _P, _I64, ctypes.POINTER(_I64), _P]),
    "gs_forward_stats": (ctypes.c_int, [ctypes.POINTER(GsOptions), _I64, _I32, ctypes.POINTER(GsCamera), _P, _SZ,
                                        ctypes.POINTER(_I64), _P]),
    "gs_tile_count": (_I64, [ctypes.POINTER(GsOptions), _I32, ctypes.POINTER(GsCamera)]),
    "gs_schedule": (ctypes.c_int, [ctypes.POINTER(GsOptions), _I64, _I32, ctypes.POINTER(GsCamera),
                                   ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "gs_activate": (ctypes.c_int, [_I64, _P, _P, _P, _P, _P]),
    "gs_activation": (ctypes.c_int, [_I64, _I32, _P, _P, _P]),
    "gs_activate_backward": (ctypes.c_int, [_I64, _P, _P, _P, _P, _P, _P, _P]),
    "gs_l1_loss": (ctypes.c_int, [_I64, _P, _P, _P, _P, _P]),
    "gs_loss_workspace_query": (ctypes.c_int, [_I32, ctypes.POINTER(GsCamera), ctypes.POINTER(_SZ)]),
    "gs_l1_dssim_loss": (ctypes.c_int, [_I32, ctypes.POINTER(GsCamera), _P, _P, ctypes.c_float, _P, _P, _P, _SZ,
                                        _P]),
    "gs_l1_dssim_loss_noalloc": (ctypes.c_int, [_I32, ctypes.POINTER(GsCamera), _P, _P, ctypes.c_float, _P, _P,
                                                _P]),
    "gs_default_backscatter_options": (None, [ctypes.POINTER(GsBackscatterOptions)]),
    "gs_backscatter_workspace_query": (ctypes.c_int, [ctypes.POINTER(GsBackscatterOptions), _I32,
                                                      ctypes.POINTER(GsCamera), ctypes.POINTER(_SZ)]),
    "gs_estimate_backscatter": (ctypes.c_int, [ctypes.POINTER(GsBackscatterOptions), _I32, ctypes.POINTER(GsCamera),
                                               _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "gs_backscatter_prior": (ctypes.c_int, [_I32, _P, _P, ctypes.c_float, _P, _P, _P]),
    "gs_mcmc_add_count": (_I64, [_I64, _I64, ctypes.c_double]),
    "gs_mcmc_workspace_query": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(_SZ)]),
    "gs_mcmc_relocate": (ctypes.c_int, [ctypes.POINTER(GsMcmcState), ctypes.c_float, _P, _P, _P, _P, _SZ, _P]),
    "gs_mcmc_add": (ctypes.c_int, [ctypes.POINTER(GsMcmcState), ctypes.POINTER(GsMcmcState), _P, _P, _P, _P, _SZ,
                                   _P]),
    "gs_mcmc_noise": (ctypes.c_int, [_I64, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float, _P]),
    "gs_adam_step": (ctypes.c_int, [ctypes.POINTER(GsAdamGroup), _I32, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _I32, _P]),
    "gs_adam_step_device": (ctypes.c_int, [ctypes.POINTER(GsAdamGroup), _I32, ctypes.c_float, ctypes.c_float,
                                           ctypes.c_float, _P, _P, _P]),
    "gs_graph_begin": (ctypes.c_int, [_P]),
    "gs_graph_end": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "gs_graph_launch": (ctypes.c_int, [_P, _P]),
    "gs_graph_destroy": (ctypes.c_int, [_P]),
    "gs_profile_marker": (ctypes.c_int, [_I32, _P]),
    "gs_timer_create": (_P, [_I32]),
    "gs_timer_destroy": (None, [_P]),
    "gs_timer_reset": (None, [_P]),
    "gs_timer_read": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(_I32)]),
}

_lib = None


def lib():
    """Load libgsplash.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2411_19588_amd/build.py "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(fn: str, rc: int) -> None:
    if rc != GS_OK:
        raise GsError(fn, rc)


def default_options() -> GsOptions:
    o = GsOptions()
    lib().gs_default_options(ctypes.byref(o))
    return o


def camera_array(cams) -> ctypes.Array:
    arr = (GsCamera * len(cams))()
    for i, c in enumerate(cams):
        R = [float(x) for x in _flat(c.R, 9)]
        t = [float(x) for x in _flat(c.t, 3)]
        arr[i] = GsCamera(int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx), float(c.cy),
                          (ctypes.c_float * 9)(*R), (ctypes.c_float * 3)(*t), float(getattr(c, "near", 0.2)))
    return arr


def _flat(x, n):
    try:
        import numpy as np
        v = np.asarray(x, dtype=np.float32).reshape(-1)
    except Exception:  # pragma: no cover
        v = list(x)
    assert len(v) == n
    return v
