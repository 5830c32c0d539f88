"""ctypes declarations of the C ABI in include/jtfs.h (argument marshalling only).

Loading fails with an ImportError when libjtfs.so has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint32, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libjtfs.so")

JTFS_OK = 0
JTFS_ERR_ARG = 1
JTFS_ERR_NOMEM = 2
JTFS_ERR_HIP = 3
JTFS_ERR_WORKSPACE = 4
JTFS_ERR_UNSUPPORTED = 5
JTFS_ERR_NONFINITE = 6

JTFS_OPT_GD = 0
JTFS_OPT_MOMENTUM_BOLD = 1
JTFS_OPT_ADAM = 2

JTFS_ZEROTH = 1
JTFS_NO_AVERAGE_LOCAL = 2
JTFS_NO_AVERAGE_LOCAL_FR = 4

JTFS_REUSE_FORWARD = 1
JTFS_SHARED_WORKSPACE = 2
JTFS_NOALLOC_SCRATCH_BYTES = 64 << 20
JTFS_N_STAGES = 19
STAGE_NAMES = ["signal_dft", "l1_wavelet", "l1_modulus_dft", "l1_average", "order1_freq", "l2_wavelet",
               "freq_fwd", "freq_pool", "freq_dP", "freq_bwd", "order1_bwd", "l1_average_adj", "dY2_dft",
               "l2_adj_gather", "dZ1_dft", "l1_adj_gather", "loss", "update", "dY2_reduce"]


class jtfs_params(ctypes.Structure):
    _fields_ = [("n", c_int64), ("J", c_int32), ("Q1", c_int32), ("Q2", c_int32), ("J_fr", c_int32),
                ("Q_fr", c_int32), ("log2_T", c_int32), ("F", c_double), ("periodic", c_int32),
                ("flags", ctypes.c_uint32), ("zeroth_weight", ctypes.c_float)]


class jtfs_path(ctypes.Structure):
    _fields_ = [("order", c_int32), ("n2", c_int32), ("n_fr", c_int32), ("spin", c_int32), ("j2", c_int32),
                ("j_fr", c_int32), ("n_lambda", c_int32), ("n_frames", c_int32), ("offset", c_int64)]


class jtfs_plan_info(ctypes.Structure):
    _fields_ = [("batch", c_int32), ("n_samples_total", c_int64), ("n_coeff_total", c_int64),
                ("ws_forward", c_size_t), ("ws_backward", c_size_t),
                ("ws_shared_forward", c_size_t), ("ws_shared_backward", c_size_t)]


class jtfs_opt(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("lr", ctypes.c_float), ("momentum", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("bold_up", ctypes.c_float),
                ("bold_down", ctypes.c_float), ("state", c_void_p)]


JTFS_N_BUCKETS = 5


class jtfs_tuning(ctypes.Structure):
    _fields_ = [("fwd_rows", c_int32), ("fwd_mt", c_int32), ("bwd_rows", c_int32), ("split_bias", c_int32),
                ("fwd_rows_k", c_int32 * JTFS_N_BUCKETS), ("bwd_rows_k", c_int32 * JTFS_N_BUCKETS)]


JTFS_DEC_MAX_LAYERS = 8


class jtfs_dec_config(ctypes.Structure):
    _fields_ = [("c_in", c_int32), ("n_frames", c_int32), ("channels", c_int32), ("kernel", c_int32),
                ("n_layers", c_int32), ("stride", c_int32 * JTFS_DEC_MAX_LAYERS), ("leak", ctypes.c_float),
                ("eps", ctypes.c_float)]


# (name, restype, argtypes) for every exported function of include/jtfs.h
SIGNATURES = [
    ("jtfs_plan", c_int32, [POINTER(jtfs_params), c_int32, POINTER(c_void_p)]),
    ("jtfs_plan_tuned", c_int32, [POINTER(jtfs_params), c_int32, POINTER(jtfs_tuning), POINTER(c_void_p)]),
    ("jtfs_autotune", c_int32, [POINTER(jtfs_params), c_int32, c_void_p, POINTER(jtfs_tuning), POINTER(c_double)]),
    ("jtfs_plan_query", c_int32, [c_void_p, POINTER(jtfs_plan_info)]),
    ("jtfs_plan_offsets", c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64)]),
    ("jtfs_plan_meta", c_int32, [c_void_p, c_int32, POINTER(jtfs_path), c_int64, POINTER(c_int64)]),
    ("jtfs_plan_filters", c_int32, [c_void_p, c_int32, c_int32, POINTER(c_double), POINTER(c_double),
                                    POINTER(c_int32), POINTER(c_int32), c_int32, POINTER(c_int32)]),
    ("jtfs_plan_sizes", c_int32, [c_void_p, c_int32, POINTER(c_int64)]),
    ("jtfs_plan_ws_region", c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int64), POINTER(c_int64)]),
    ("jtfs_plan_cost", c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    ("jtfs_opt_state_floats", c_int64, [c_void_p, c_int32]),
    ("jtfs_forward", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("jtfs_forward_ex", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_uint32, c_void_p]),
    ("jtfs_plan_prepare", c_int32, [c_void_p]),
    ("jtfs_forward_noalloc", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    ("jtfs_colored_noise", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("jtfs_backward", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_uint32, c_void_p]),
    ("jtfs_metamer_step", c_int32, [c_void_p, c_void_p, c_void_p, POINTER(jtfs_opt), c_void_p, c_void_p, c_size_t,
                                    c_void_p]),
    ("jtfs_joint_wavelet", c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    ("jtfs_opt_status", c_int32, [c_void_p, POINTER(jtfs_opt), POINTER(c_int32), c_void_p]),
    ("jtfs_loss", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, ctypes.c_float, c_void_p]),
    ("jtfs_timing_enable", c_int32, [c_void_p, c_int32]),
    ("jtfs_timing_stages", c_int32, [c_void_p, c_uint32]),
    ("jtfs_timing_read", c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64), c_int32]),
    ("jtfs_plan_destroy", None, [c_void_p]),
    ("jtfs_dec_create", c_int32, [POINTER(jtfs_dec_config), c_int32, POINTER(c_void_p)]),
    ("jtfs_dec_query", c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_size_t)]),
    ("jtfs_dec_forward", c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("jtfs_dec_backward", c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("jtfs_dec_adam_step", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_float, c_void_p]),
    ("jtfs_dec_ws_region", c_int32, [c_void_p, c_int32, c_int32, POINTER(c_size_t), POINTER(c_size_t)]),
    ("jtfs_dec_destroy", None, [c_void_p]),
    ("jtfs_status_str", c_char_p, [c_int32]),
    ("jtfs_last_error", c_char_p, []),
]

_lib = None


def lib():
    """The loaded library (loaded once)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_2602_11896_amd.build)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class JTFSError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        detail = L.jtfs_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.jtfs_status_str(status).decode()} ({status}): {detail}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != JTFS_OK:
        raise JTFSError(status, where)
