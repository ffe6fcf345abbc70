"""ctypes binding of the C ABI declared in include/ridge_detect.h (argument marshalling only).

Loading fails loudly if the HIP library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libridgedetect.so")

RD_OK, RD_E_INVALID, RD_E_NOMEM, RD_E_DEVICE, RD_E_TOO_LARGE, RD_E_TRUNCATED, RD_E_OVERFLOW = range(7)
RD_U16, RD_F32 = 1, 2


class RdFrame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("pitch_bytes", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("on_device", ctypes.c_int32), ("data", ctypes.c_void_p)]


class RdParams(ctypes.Structure):
    _fields_ = [("sigma_smooth", ctypes.c_float), ("k_threshold", ctypes.c_float),
                ("r_min", ctypes.c_int32), ("r_max", ctypes.c_int32),
                ("vote_threshold", ctypes.c_int32), ("peak_fraction", ctypes.c_float),
                ("sig_slope", ctypes.c_float), ("sig_icpt", ctypes.c_float),
                ("annulus_halfwidth", ctypes.c_int32), ("min_fit_points", ctypes.c_int32),
                ("measure", ctypes.c_int32), ("r_step", ctypes.c_int32), ("curvature_fp32", ctypes.c_int32)]


class RdRing(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_float), ("cy", ctypes.c_float), ("r", ctypes.c_float),
                ("score", ctypes.c_float), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("r_bin", ctypes.c_int32), ("n_fit", ctypes.c_int32), ("fit_ok", ctypes.c_int32)]


class RdCreateInfo(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_width", ctypes.c_int32), ("max_height", ctypes.c_int32),
                ("max_peaks", ctypes.c_int32), ("max_frames", ctypes.c_int32),
                ("max_batch_pixels", ctypes.c_int64), ("stream", ctypes.c_void_p)]


class RdTuning(ctypes.Structure):
    _fields_ = [("stencil_tile", ctypes.c_int32), ("vote_lds_kb", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class RdLinkParams(ctypes.Structure):
    _fields_ = [("gate", ctypes.c_float), ("memory", ctypes.c_int32), ("depth_c0", ctypes.c_double),
                ("depth_c1", ctypes.c_double), ("depth_c2", ctypes.c_double), ("model", ctypes.c_int32)]


class RdError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64

# name -> (restype, argtypes); every function of the header is listed here
SIGNATURES = {
    "rd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rd_validate_params": (ctypes.c_int, [_P(RdParams)]),
    "rd_level_tables": (ctypes.c_int, [_P(RdParams), _i32, _vp, _vp, _vp]),
    "rd_validate_ridges": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32]),
    "rd_create": (ctypes.c_int, [_P(RdCreateInfo), _P(_vp)]),
    "rd_destroy": (None, [_vp]),
    "rd_detect": (ctypes.c_int, [_vp, _P(RdFrame), _P(RdParams), _P(RdRing), _i32, _P(_i32)]),
    "rd_detect_batch": (ctypes.c_int, [_vp, _P(RdFrame), _i32, _P(RdParams), _P(RdRing), _P(_i64), _P(_i32),
                                       _P(_i32)]),
    "rd_set_tuning": (ctypes.c_int, [_vp, _P(RdTuning)]),
    "rd_get_tuning": (ctypes.c_int, [_vp, _P(RdTuning)]),
    "rd_autotune": (ctypes.c_int, [_vp, _P(RdFrame), _i32, _P(RdParams), _i32, _P(RdTuning)]),
    "rd_read_stats": (ctypes.c_int, [_vp, _P(_i64)]),
    "rd_enable_timing": (ctypes.c_int, [_vp, _i32]),
    "rd_read_timing": (ctypes.c_int, [_vp, _vp, _vp, _i32]),
    "rd_measure_lds_atomics": (ctypes.c_int, [_i32, _i32, _P(ctypes.c_double), _P(ctypes.c_double)]),
    "rd_stage_curvature": (ctypes.c_int, [_vp, _P(RdFrame), _P(RdParams), _vp, _vp]),
    "rd_stage_ridges": (ctypes.c_int, [_vp, _P(RdFrame), _P(RdParams), _vp, _vp, _vp, _i64, _P(_i64)]),
    "rd_stage_accumulate": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _P(RdParams), _vp, _vp]),
    "rd_detect_ridges": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _P(RdParams), _P(RdRing), _i32,
                                        _P(_i32)]),
    "rd_encode_ridges": (ctypes.c_int, [_vp, _P(RdFrame), _i32, _P(RdParams), _vp, _i64, _P(_i64)]),
    "rd_detect_encoded": (ctypes.c_int, [_vp, _vp, _i32, _P(_i64), _i32, _P(RdParams), _P(RdRing), _P(_i64),
                                         _P(_i32), _P(_i32)]),
    "rd_detect_noalloc": (ctypes.c_int, [_P(RdFrame), _P(RdParams), _vp, _vp, _i32, _P(_i32)]),
    "rd_soft_ridges": (ctypes.c_int, [_vp, _P(RdFrame), _P(RdParams), _vp, _vp, _i64, _P(_i64)]),
    "rd_soft_forward": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _P(RdParams), _vp]),
    "rd_soft_backward": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _P(RdParams), _vp, _vp, _P(_i64)]),
    "rd_hessian_backward": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _P(RdParams), _vp]),
    "rd_fit_loss": (ctypes.c_int, [_vp, _P(RdFrame), _vp, _vp, _i64, ctypes.c_double, _vp, _vp]),
    "rd_fit_loss_backward": (ctypes.c_int, [_vp, _P(RdFrame), _vp, _vp, _i64, ctypes.c_double, _vp, _vp, _vp]),
    "rd_profile_vote_phases": (ctypes.c_int, [_vp, _P(RdFrame), _P(RdParams), _vp]),
    "rd_profile_vote_tiles": (ctypes.c_int, [_vp, _P(RdFrame), _P(RdParams), _vp, ctypes.c_int32, _P(ctypes.c_int32)]),
    "rd_soft_ridges_batch": (ctypes.c_int, [_vp, _P(RdFrame), _i32, _P(RdParams), _vp, _vp, _i64, _vp]),
    "rd_soft_forward_batch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _P(RdParams), _vp]),
    "rd_soft_backward_batch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _P(RdParams), _vp, _vp,
                                              _P(_i64)]),
    "rd_hessian_backward_batch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _P(RdParams), _vp]),
    "rd_fit_loss_batch": (ctypes.c_int, [_vp, _P(RdFrame), _i32, _vp, _vp, _vp, _i64, ctypes.c_double, _vp, _vp]),
    "rd_fit_loss_backward_batch": (ctypes.c_int, [_vp, _P(RdFrame), _i32, _vp, _vp, _vp, _i64, ctypes.c_double,
                                                  _vp, _vp, _vp]),
    "rd_refine": (ctypes.c_int, [_vp, _P(RdFrame), _i32, _vp, _vp, _i64, ctypes.c_double, _i32, ctypes.c_double,
                                 _vp, _vp, _vp]),
    "rd_linker_create": (ctypes.c_int, [_P(RdLinkParams), _i32, _i32, _vp, _P(_vp)]),
    "rd_linker_destroy": (None, [_vp]),
    "rd_linker_reset": (ctypes.c_int, [_vp]),
    "rd_linker_info": (ctypes.c_int, [_vp, _P(_i32), _P(_i32), _P(_i32)]),
    "rd_link": (ctypes.c_int, [_vp, _vp, _P(_i32), _i32, _vp, _vp]),
}

_lib = None


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library {LIB_PATH} is not built; run `python -m paper_1310_1371_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().rd_status_string(status).decode()
    except ImportError:
        return "library not loaded"


def check(status: int, what: str, ok=(RD_OK,)):
    if status not in ok:
        raise RdError(status, what)
    return status


def make_params(d: dict) -> RdParams:
    return RdParams(float(d["sigma_smooth"]), float(d["k_threshold"]), int(d["r_min"]), int(d["r_max"]),
                    int(d["vote_threshold"]), float(d["peak_fraction"]), float(d["sig_slope"]),
                    float(d["sig_icpt"]), int(d["annulus_halfwidth"]), int(d["min_fit_points"]),
                    int(d.get("measure", 0)), int(d.get("r_step", 1)), int(d.get("curvature_fp32", 0)))


def n_levels(d: dict) -> int:
    """Accumulator levels of a parameter set: (r_max - r_min) / r_step + 3."""
    s = max(int(d.get("r_step", 1)), 1)
    return (int(d["r_max"]) - int(d["r_min"])) // s + 3
