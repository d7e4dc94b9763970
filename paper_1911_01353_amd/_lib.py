"""ctypes declarations of ``include/jerk.h`` (argument marshalling only).

The shared library is loaded from this package's directory. There is no
fallback: if ``libjerk.so`` is missing the import of the binding fails with a
message saying how to build it.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# JERK_LIBRARY selects another build of the same library (the host-sanitized libjerk_asan.so)
LIB_PATH = os.environ.get("JERK_LIBRARY") or os.path.join(HERE, "libjerk.so")

JERK_OK = 0
JERK_EINVAL = -1
JERK_ENOMEM = -2
JERK_EAGAIN = -3
JERK_EPENDING = -4
JERK_EHIP = -5
JERK_EUNSUPPORTED = -6
JERK_EINTERNAL = -7
JERK_ECANCELED = -8
NOALLOC_MAX_ROWS = 32768  # JERK_NOALLOC_MAX_ROWS

PATH_FFT_FP32 = 0
PATH_GEMM_SPLIT_BF16 = 1
PATH_GEMM_FP16 = 2
PATH_AUTO = 3
PATH_NAMES = {"fft": PATH_FFT_FP32, "split_bf16": PATH_GEMM_SPLIT_BF16, "fp16": PATH_GEMM_FP16,
              "auto": PATH_AUTO}


class PlanDesc(C.Structure):
    _fields_ = [
        ("nbins", C.c_int64),
        ("zmax", C.c_double), ("wmax", C.c_double), ("dz", C.c_double), ("dw", C.c_double),
        ("numbetween", C.c_int32), ("margin_bins", C.c_int32), ("path", C.c_int32),
        ("seg_len", C.c_int32), ("templates_per_block", C.c_int32), ("tap_quantum", C.c_int32),
        ("flags", C.c_uint32),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("n_z", C.c_int32), ("n_w", C.c_int32), ("n_templates", C.c_int32), ("n_groups", C.c_int32),
        ("nbins", C.c_int64), ("n_r", C.c_int64),
        ("max_taps", C.c_int32), ("path", C.c_int32),
        ("bank_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t), ("plane_row_bytes", C.c_size_t),
        ("taps_offset", C.c_size_t),
    ]


class GroupInfo(C.Structure):
    _fields_ = [
        ("taps", C.c_int32), ("seg_len", C.c_int32), ("templates_per_block", C.c_int32),
        ("path", C.c_int32), ("n_members", C.c_int32), ("first_member", C.c_int32),
        ("fft_ept", C.c_int32), ("reserved", C.c_int32), ("taps_offset", C.c_size_t),
    ]


class BatchItem(C.Structure):
    _fields_ = [
        ("spec", C.c_void_p), ("nbins", C.c_int64), ("plane", C.c_void_p), ("ld", C.c_int64),
        ("peaks", C.c_void_p), ("keys_ld", C.c_int64),
    ]


class BatchCandItem(C.Structure):
    _fields_ = [
        ("spec", C.c_void_p), ("nbins", C.c_int64), ("out", C.c_void_p), ("capacity", C.c_int64),
        ("count", C.c_void_p), ("stats", C.c_void_p),
    ]


class Peak(C.Structure):
    _fields_ = [("power", C.c_float), ("p", C.c_uint32)]


BATCH_GRAPH = 1
BATCH_FLAT = 2
BATCH_PERSISTENT = 4
SERVE_DRYRUN = 1


class ServeDesc(C.Structure):
    _fields_ = [
        ("max_active", C.c_int32), ("queue_capacity", C.c_int32), ("tiles_per_launch", C.c_int64),
        ("seg_len", C.c_int32), ("slots", C.c_int32), ("flags", C.c_uint32), ("reserved", C.c_int32),
    ]


class Request(C.Structure):
    _fields_ = [
        ("spec", C.c_void_p), ("nbins", C.c_int64),
        ("zmax", C.c_double), ("wmax", C.c_double), ("dz", C.c_double), ("dw", C.c_double),
        ("path", C.c_int32), ("peaks_capacity", C.c_int32),
        ("plane", C.c_void_p), ("ld", C.c_int64), ("peaks", C.c_void_p),
        ("top", C.c_void_p), ("top_capacity", C.c_int32), ("reserved", C.c_int32),
    ]


class Top(C.Structure):
    _fields_ = [("t", C.c_int32), ("p", C.c_uint32), ("power", C.c_float), ("reserved", C.c_int32)]


class Result(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("n_templates", C.c_int32), ("best_power", C.c_float), ("best_t", C.c_int32),
        ("best_p", C.c_uint32), ("top_count", C.c_int32), ("points", C.c_uint64),
        ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_first_launch", C.c_double), ("t_done", C.c_double),
    ]


class ServeStats(C.Structure):
    _fields_ = [
        ("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64), ("launches", C.c_uint64),
        ("bank_builds", C.c_uint64), ("bank_evictions", C.c_uint64), ("queued", C.c_int32), ("active", C.c_int32),
        ("arena_used", C.c_size_t), ("arena_bytes", C.c_size_t),
        ("shared_launches", C.c_uint64), ("max_in_flight", C.c_int32), ("reserved", C.c_int32),
    ]

# name -> (restype, argtypes)
SIGNATURES = {
    "jerk_status_str": (C.c_char_p, [C.c_int32]),
    "jerk_last_error": (C.c_char_p, []),
    "jerk_version": (C.c_char_p, []),
    "jerk_plan_create": (C.c_int32, [C.POINTER(PlanDesc), C.POINTER(C.c_void_p)]),
    "jerk_plan_destroy": (C.c_int32, [C.c_void_p]),
    "jerk_plan_info": (C.c_int32, [C.c_void_p, C.POINTER(PlanInfo)]),
    "jerk_plan_group": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(GroupInfo)]),
    "jerk_plan_template": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "jerk_plan_members": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32]),
    "jerk_plan_set_group": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "jerk_templates_build": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "jerk_search": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "jerk_search_group": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                      C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "jerk_search_members": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                        C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "jerk_batch_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32]),
    "jerk_batch_keys_per_row": (C.c_int64, [C.c_void_p, C.c_int64]),
    "jerk_batch_search": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(BatchItem), C.c_int32, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_size_t, C.c_uint32, C.c_void_p]),
    "jerk_peaks_reduce": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "jerk_stats_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int64]),
    "jerk_stream_check": (C.c_int32, [C.c_void_p]),
    "jerk_spectrum_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "jerk_harmonic_shape": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "jerk_harmonic_sum": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_void_p, C.c_int64,
                                      C.c_void_p]),
    "jerk_spectrum_prepare": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "jerk_plane_stats": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_size_t, C.c_void_p]),
    "jerk_find_candidates": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_void_p, C.c_double,
                                         C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "jerk_batch_search_candidates_workspace_bytes": (C.c_size_t, [C.c_void_p, C.POINTER(BatchCandItem), C.c_int32,
                                                                  C.c_int32, C.c_int32, C.c_double, C.c_int64]),
    "jerk_batch_search_candidates": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(BatchCandItem), C.c_int32, C.c_int32,
                                                  C.c_int32, C.c_double, C.c_double, C.c_int64, C.c_void_p, C.c_size_t,
                                                  C.c_void_p]),
    "jerk_search_peaks_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32, C.c_int32]),
    "jerk_search_peaks_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                              C.c_void_p, C.c_void_p]),
    "jerk_search_peaks": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                                      C.c_void_p, C.c_size_t, C.c_void_p]),
    "jerk_search_candidates_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_double,
                                                            C.c_int64]),
    "jerk_search_candidates": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                           C.c_double, C.c_double, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                           C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "jerk_serve_create": (C.c_int32, [C.POINTER(ServeDesc), C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    "jerk_serve_submit": (C.c_int32, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "jerk_serve_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(Result)]),
    "jerk_serve_wait": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(Result), C.c_double]),
    "jerk_serve_stats_get": (C.c_int32, [C.c_void_p, C.POINTER(ServeStats)]),
    "jerk_serve_inject_failure": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int64]),
    "jerk_serve_destroy": (C.c_int32, [C.c_void_p]),
    "jerk_autotune_scratch_bytes": (C.c_size_t, [C.c_void_p, C.c_int64]),
    "jerk_plan_autotune": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t, C.c_uint32,
                                       C.c_void_p]),
}

TUNE_UNIFORM = 1

_lib = None


class JerkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_str(status)} ({status}): {msg}")
        self.status = status


def load() -> C.CDLL:
    """Load ``libjerk.so`` (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_1911_01353_amd.build` "
                          "(the HIP library is required; there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_str(status: int) -> str:
    return load().jerk_status_str(status).decode()


def check(status: int) -> None:
    if status != JERK_OK:
        msg = load().jerk_last_error().decode()
        raise JerkError(status, msg)
