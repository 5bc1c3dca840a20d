"""ctypes binding of libhk.so (argument marshalling only).

The library is built in-tree by ``paper_1405_1931_amd/build.py`` (or
``__graft_entry__.build()``).  There is no fallback: if the shared library is
missing, loading raises, so a GPU run can never silently take another path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhk.so")
HEADER = os.path.join(HERE, "..", "include", "hk.h")

HK_OK = 0
HK_ERR_INVALID_ARG = -1
HK_ERR_TOO_LARGE = -2
HK_ERR_NO_WORKSPACE = -3
HK_ERR_HIP = -4
HK_ERR_DEVICE = -5
HK_ERR_TIMEOUT = -6
HK_PRED_GT, HK_PRED_EQ, HK_PRED_U8 = 0, 1, 2


class HkJob(ctypes.Structure):
    _fields_ = [
        ("phi", ctypes.c_void_p),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("periodic_mask", ctypes.c_uint32),
        ("labels", ctypes.c_void_p),
        ("n_clusters", ctypes.c_void_p),
        ("sizes", ctypes.c_void_p),
    ]


class HkServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("batches", ctypes.c_int64),
        ("mean_batch_jobs", ctypes.c_double),
        ("pending", ctypes.c_int64),
        ("running", ctypes.c_int64),
        ("sites_completed", ctypes.c_int64),
        ("arena_bytes", ctypes.c_int64),
        ("arena_in_use", ctypes.c_int64),
        ("arena_peak", ctypes.c_int64),
        ("latency_samples", ctypes.c_int64),
        ("latency_p50_ns", ctypes.c_int64),
        ("latency_p99_ns", ctypes.c_int64),
        ("latency_max_ns", ctypes.c_int64),
        ("latency_mean_ns", ctypes.c_double),
        ("span_ns", ctypes.c_int64),
    ]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64

_SIGS = {
    "hk_label": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hk_label_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "hk_label_pred": (ctypes.c_int, [_P, _I32, ctypes.c_float, _I32, _I32, _I32, ctypes.c_uint32, _P, _P, _P, _P]),
    "hk_incr_create": (ctypes.c_int, [_I32, _I32, _I32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "hk_incr_label": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "hk_incr_device_error": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "hk_incr_destroy": (None, [_P]),
    "hk_label_batched": (ctypes.c_int, [ctypes.POINTER(HkJob), ctypes.c_int32, ctypes.c_void_p]),
    "hk_max_clusters": (ctypes.c_int64, [ctypes.c_int32] * 3),
    "hk_workspace_bytes": (ctypes.c_int64, [ctypes.c_int32] * 3),
    "hk_batched_workspace_bytes": (ctypes.c_int64, [ctypes.POINTER(HkJob), ctypes.c_int32]),
    "hk_reserve": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p]),
    "hk_release": (None, []),
    "hk_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "hk_set_brick": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32]),
    "hk_get_brick": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "hk_set_brick_for_shape": (ctypes.c_int, [ctypes.c_int32] * 5),
    "hk_device_error": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "hk_debug_counters": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "hk_profile_enable": (ctypes.c_int, [ctypes.c_int32]),
    "hk_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]),
    "hk_phase_count": (ctypes.c_int32, []),
    "hk_phase_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "hk_classify": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, ctypes.c_uint32, _P, _P, _P, _P, _P]),
    "hk_droplet_stats": (ctypes.c_int, [_P, _P, _I64, _I64, ctypes.c_double, _I32, _P, _P, _P, _P]),
    "hk_label_droplets": (ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.c_uint32, _P, _P, _P, _I64, ctypes.c_double, _I32,
                                         _P, _P, _P, _P]),
    "hk_autotune": (ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.c_uint32, _P, _P, _P, _I32, _P,
                                   ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float)]),
    "hk_autotune_batched": (ctypes.c_int, [ctypes.POINTER(HkJob), _I32, _I32, _P, ctypes.POINTER(_I32),
                                           ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float)]),
    "hk_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "hk_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "hk_server_create": (ctypes.c_int, [_I64, _I32, _I32, ctypes.POINTER(_P)]),
    "hk_server_create_simulated": (ctypes.c_int, [_I64, _I32, _I32, _I64, ctypes.c_double, ctypes.POINTER(_P)]),
    "hk_server_footprint": (_I64, [_I32, _I32, _I32]),
    "hk_server_now_ns": (_I64, []),
    "hk_server_submit": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, ctypes.c_uint32, _I64,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "hk_server_submit_after": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, ctypes.c_uint32, _I64, _P,
                                              ctypes.POINTER(ctypes.c_uint64)]),
    "hk_server_sim_fail": (ctypes.c_int, [_P, ctypes.c_uint64, _I32]),
    "hk_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "hk_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, _I64]),
    "hk_server_drain": (ctypes.c_int, [_P, _I64]),
    "hk_server_result": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(_P), ctypes.POINTER(_I64),
                                        ctypes.POINTER(_P), ctypes.POINTER(_I64)]),
    "hk_server_release": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "hk_server_read_stats": (ctypes.c_int, [_P, ctypes.POINTER(HkServerStats)]),
    "hk_server_reset_stats": (ctypes.c_int, [_P]),
    "hk_server_destroy": (ctypes.c_int, [_P]),
}

_lib = None


def load(path: str | None = None):
    """Load libhk.so (LIB_PATH, read at the first call); raises RuntimeError
    if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library {path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)  # every declared entry point must be exported
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HkError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.hk_status_string(status).decode()
        super().__init__(f"{where}: {msg} ({status})")
        self.status = status


def check(status: int, where: str):
    if status != HK_OK:
        raise HkError(status, where)
