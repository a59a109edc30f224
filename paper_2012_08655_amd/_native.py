"""ctypes view of the C ABI in include/foveate.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfoveate.so")

FOV_OK, FOV_EINVAL, FOV_EDTYPE, FOV_ELAYOUT, FOV_EALIAS = 0, -1, -2, -3, -4
FOV_ENOMEM, FOV_EAGAIN, FOV_EHIP, FOV_ECLOSED, FOV_ENOTICKET, FOV_ERANGE = -5, -6, -7, -8, -9, -10
STATUS_NAMES = {0: "FOV_OK", -1: "FOV_EINVAL", -2: "FOV_EDTYPE", -3: "FOV_ELAYOUT", -4: "FOV_EALIAS",
                -5: "FOV_ENOMEM", -6: "FOV_EAGAIN", -7: "FOV_EHIP", -8: "FOV_ECLOSED",
                -9: "FOV_ENOTICKET", -10: "FOV_ERANGE"}
FOV_U8, FOV_F32, FOV_F64 = 0, 1, 2


class FovTensor(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("n", ctypes.c_int32), ("c", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("sn", ctypes.c_int64), ("sc", ctypes.c_int64), ("sh", ctypes.c_int64), ("sw", ctypes.c_int64)]


class FovParams(ctypes.Structure):
    _fields_ = [("fix_x", ctypes.c_double), ("fix_y", ctypes.c_double), ("e0", ctypes.c_double),
                ("slope", ctypes.c_double), ("cap", ctypes.c_double), ("block", ctypes.c_int32),
                ("origin_x", ctypes.c_int32), ("origin_y", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sigma_map", ctypes.c_void_p)]


class FovServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_batch_frames", ctypes.c_int32),
                ("max_inflight_batches", ctypes.c_int32), ("max_requests", ctypes.c_int32),
                ("in_dtype", ctypes.c_int32), ("out_dtype", ctypes.c_int32), ("max_fragments", ctypes.c_int32),
                ("max_block", ctypes.c_int32), ("max_sigma", ctypes.c_double), ("use_graph", ctypes.c_int32),
                ("test_fake_device_us", ctypes.c_int32), ("test_fail_every", ctypes.c_int32),
                ("shared_stream", ctypes.c_int32)]


class FovTiming(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double), ("batch_frames", ctypes.c_int32), ("status", ctypes.c_int32)]


class FovTuning(ctypes.Structure):
    _fields_ = [("split", ctypes.c_int32), ("strip_rows", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("merge", ctypes.c_int32), ("chan_split", ctypes.c_int32), ("time_us", ctypes.c_float)]


# Every symbol declared in include/foveate.h, with (restype, argtypes).
_TP = ctypes.POINTER(FovTensor)
_PP = ctypes.POINTER(FovParams)
_I32P = ctypes.POINTER(ctypes.c_int32)
SIGNATURES = {
    "foveate_grid": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _PP, _I32P, _I32P]),
    "foveate_plan": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _PP, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "foveate_csf_params": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, _PP]),
    "foveate_fragment_shift": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int32, _I32P, _I32P]),
    "foveate_plan_host": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _PP, ctypes.c_void_p, ctypes.c_void_p]),
    "foveate_forward": (ctypes.c_int, [_TP, _TP, _PP, ctypes.c_int32, ctypes.c_void_p]),
    "foveate_forward_batch": (ctypes.c_int, [_TP, _TP, _PP, ctypes.c_int32, ctypes.c_void_p]),
    "foveate_forward_noalloc": (ctypes.c_int, [_TP, _TP, _PP, ctypes.c_int32, ctypes.c_void_p]),
    "foveate_backward": (ctypes.c_int, [_TP, _TP, _PP, ctypes.c_int32, ctypes.c_void_p]),
    "foveate_autotune": (ctypes.c_int, [_TP, _TP, _PP, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.POINTER(FovTuning)]),
    "foveate_autotune_batch": (ctypes.c_int, [_TP, _TP, _PP, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.POINTER(FovTuning)]),
    "foveate_tuning_force": (ctypes.c_int, [ctypes.POINTER(FovTuning)]),
    "foveate_tuning_clear": (ctypes.c_int, []),
    "foveate_tuning_count": (ctypes.c_int, [_I32P]),
    "foveate_tuning_save": (ctypes.c_int, [ctypes.c_char_p]),
    "foveate_tuning_load": (ctypes.c_int, [ctypes.c_char_p]),
    "foveate_profile_begin": (ctypes.c_int, [ctypes.c_int32]),
    "foveate_profile_end": (ctypes.c_int, [ctypes.POINTER(ctypes.c_float), ctypes.c_int32, _I32P]),
    "foveate_profile_every": (ctypes.c_int, [ctypes.c_int32]),
    "foveate_now": (ctypes.c_double, []),
    "foveate_stream_timestamp": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "foveate_server_create": (ctypes.c_int, [ctypes.POINTER(FovServerCfg), ctypes.POINTER(ctypes.c_void_p)]),
    "foveate_submit": (ctypes.c_int, [ctypes.c_void_p, _TP, _TP, _PP, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_uint64)]),
    "foveate_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, _I32P, ctypes.POINTER(FovTiming)]),
    "foveate_server_drain": (ctypes.c_int, [ctypes.c_void_p]),
    "foveate_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "foveate_pipeline_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_size_t, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_void_p)]),
    "foveate_pipeline_submit": (ctypes.c_int, [ctypes.c_void_p, _TP, _TP, _PP, ctypes.POINTER(ctypes.c_uint64)]),
    "foveate_pipeline_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, _I32P]),
    "foveate_pipeline_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "foveate_pipeline_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "foveate_last_error": (ctypes.c_char_p, []),
    "foveate_version": (ctypes.c_char_p, []),
}

_lib = None


class FoveateError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


def lib():
    """Load libfoveate.so; raises if it has not been built (no fallback).

    PyTorch, when installed, is imported first: it brings its own HIP runtime,
    and the library must resolve its HIP symbols against that same runtime
    (device pointers and streams come from PyTorch).  Loading the library
    first would pull the system runtime in beside PyTorch's.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfoveate.so is not built (run paper_2012_08655_amd._build.build()); "
                              "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != FOV_OK:
        raise FoveateError(status, lib().foveate_last_error().decode())
    return status


def make_params(p, sigma_map_ptr=None) -> FovParams:
    return FovParams(float(p["fix_x"]), float(p["fix_y"]), float(p["e0"]), float(p["slope"]), float(p["cap"]),
                     int(p.get("block", 32)), int(p.get("origin_x", 0)), int(p.get("origin_y", 0)), 0,
                     sigma_map_ptr)
