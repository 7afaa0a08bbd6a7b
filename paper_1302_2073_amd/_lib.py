"""ctypes binding of libprost.so (argument marshalling only).

Every entry point of include/prost.h is exposed under the same name.  The
library must exist (built by paper_1302_2073_amd.build); there is no
fallback path: importing the functions without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprost.so")

PROS_OK = 0
PROS_EINVAL = -1
PROS_ENOMEM = -2
PROS_EHIP = -3
PROS_ESTATE = -4
PROS_EBADFRAME = -5
PROS_ETIMEOUT = -6
PROS_EUNSUPPORTED = -7
PROS_LPCOST_SCRATCH_BYTES = 8 << 20   # fixed scratch of pros_lpcost_bwd_noalloc (include/prost.h)

PROS_F32 = 0
PROS_BF16 = 1
PROS_COST_LP = 0
PROS_COST_LOG = 1
PROS_MAX_K = 16
PROS_MAX_CG = 16


class pros_params(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32), ("channels", C.c_int32),
        ("k", C.c_int32), ("cg_iters", C.c_int32), ("cost", C.c_int32),
        ("p", C.c_double), ("mu", C.c_double), ("delta", C.c_double), ("omega", C.c_double),
        ("t_init", C.c_double), ("t_min", C.c_double), ("i_init", C.c_int32),
        ("storage", C.c_int32), ("reorth_every", C.c_int32),
        ("labels_after_update", C.c_int32), ("weights_from_filtered", C.c_int32),
        ("preprocess", C.c_int32),
        ("ysolve", C.c_int32),
        ("seed", C.c_uint64),
    ]


class pros_stats(C.Structure):
    _fields_ = [
        ("frame", C.c_int64), ("cg_steps", C.c_int32), ("restarts", C.c_int32),
        ("updated", C.c_int32), ("bad_frame", C.c_int32),
        ("f", C.c_double * (PROS_MAX_CG + 1)), ("alpha", C.c_double * PROS_MAX_CG),
        ("beta", C.c_double * PROS_MAX_CG),
        ("t", C.c_double), ("sigma", C.c_double), ("theta", C.c_double),
        ("zeta", C.c_double), ("nu", C.c_double), ("fg_pixels", C.c_int64),
    ]


class pros_launch_info(C.Structure):
    _fields_ = [("workgroups", C.c_int32), ("threads", C.c_int32), ("rows_per_thread", C.c_int32),
                ("pixels_per_wg", C.c_int32), ("barriers_per_frame", C.c_int32), ("sync_mode", C.c_int32),
                ("curvature", C.c_int32)]


class pros_batch_config(C.Structure):
    _fields_ = [("register_budget", C.c_int32), ("workgroups_per_cu", C.c_int32), ("tile_scale", C.c_double),
                ("strategy", C.c_int32), ("sync_mode", C.c_int32), ("workgroups", C.c_int32),
                ("rounds", C.c_int32), ("threads", C.c_int32)]


class ProstError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = status
        super().__init__(f"{strerror(status)} ({status}): {detail}")


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "pros_params_default": (C.c_int, [C.POINTER(pros_params), C.c_int32, C.c_int32, C.c_int32]),
    "pros_validate": (C.c_int, [C.POINTER(pros_params)]),
    "pros_init": (C.c_int, [C.POINTER(pros_params), C.c_void_p, C.POINTER(C.c_void_p)]),
    "pros_destroy": (None, [C.c_void_p]),
    "pros_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "pros_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]),
    "pros_track_frame": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    "pros_track_frames": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_int32, C.c_int32]),
    "pros_get_mask": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    "pros_get_stats": (C.c_int, [C.c_void_p, C.POINTER(pros_stats)]),
    "pros_sync": (C.c_int, [C.c_void_p]),
    "pros_reorthonormalize": (C.c_int, [C.c_void_p]),
    "pros_get_launch_info": (C.c_int, [C.c_void_p, C.POINTER(pros_launch_info)]),
    "pros_set_launch": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "pros_set_curvature": (C.c_int, [C.c_void_p, C.c_int32]),
    "pros_set_dispatch": (C.c_int, [C.c_void_p, C.c_int32]),
    "pros_batch_set_dispatch": (C.c_int, [C.c_void_p, C.c_int32]),
    "pros_debug_trace": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pros_set_preprocess": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "pros_set_score_output": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pros_quality_counts": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "pros_roc_counts": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                  C.c_void_p, C.c_void_p]),
    "pros_get_preprocess": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pros_resample_rgb8": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_void_p, C.c_int32,
                                     C.c_int32, C.c_int32, C.c_double, C.c_void_p]),
    "pros_mask_upsample": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                     C.c_void_p]),
    "pros_ingest_init": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                   C.POINTER(C.c_void_p)]),
    "pros_ingest_slot": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "pros_ingest_submit": (C.c_int, [C.c_void_p]),
    "pros_ingest_push": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pros_ingest_mask": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    "pros_ingest_destroy": (None, [C.c_void_p]),
    "pros_batch_init": (C.c_int, [C.POINTER(pros_params), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pros_batch_destroy": (None, [C.c_void_p]),
    "pros_batch_set_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "pros_batch_get_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.POINTER(C.c_int64)]),
    "pros_batch_set_preprocess": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64]),
    "pros_batch_get_preprocess": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
    "pros_batch_set_frames": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_int32]),
    "pros_batch_track": (C.c_int, [C.c_void_p]),
    "pros_batch_track_frames": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "pros_batch_track_steps": (C.c_int, [C.c_void_p, C.c_int32]),
    "pros_batch_use_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "pros_batch_sync": (C.c_int, [C.c_void_p]),
    "pros_batch_get_mask": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32]),
    "pros_batch_get_stats": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(pros_stats)]),
    "pros_batch_reorthonormalize": (C.c_int, [C.c_void_p]),
    "pros_batch_get_config": (C.c_int, [C.c_void_p, C.POINTER(pros_batch_config)]),
    "pros_batch_configure": (C.c_int, [C.c_void_p, C.POINTER(pros_batch_config)]),
    "pros_batch_tune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(pros_batch_config), C.POINTER(C.c_double)]),
    "pros_lpcost_workspace_size": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "pros_lpcost_fwd": (C.c_int, [C.c_void_p] * 5 + [C.c_int32] * 4 + [C.c_float]
                        + [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "pros_lpcost_bwd": (C.c_int, [C.c_void_p] * 5 + [C.c_int32] * 4 + [C.c_float]
                        + [C.c_void_p] * 5 + [C.c_void_p, C.c_size_t, C.c_void_p]),
    "pros_lpcost_bwd_noalloc": (C.c_int, [C.c_void_p] * 5 + [C.c_int32] * 4 + [C.c_float]
                                + [C.c_void_p] * 5 + [C.c_void_p]),
    "pros_random_subspace": (C.c_int, [C.c_uint64, C.c_uint32, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p]),
    "pros_strerror": (C.c_char_p, [C.c_int]),
    "pros_last_error": (C.c_char_p, []),
}


def lib():
    """Load libprost.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1302_2073_amd.build`")
        # torch first: its libraries bring their own HIP runtime under the
        # same soname as the system one, and the library must bind to the
        # runtime that owns torch's device memory and streams (loaded the
        # other way round, the first launch finds no device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def strerror(status):
    try:
        return lib().pros_strerror(int(status)).decode()
    except ImportError:
        return f"status {status}"


def last_error():
    return lib().pros_last_error().decode()


def check(status, allow=()):
    if status != PROS_OK and status not in allow:
        raise ProstError(status, last_error())
    return status


def __getattr__(name):
    if name in _SIGS:
        return getattr(lib(), name)
    raise AttributeError(name)
