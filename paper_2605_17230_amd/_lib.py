"""ctypes binding of libtnmld.so (argument marshalling only).

Every entry point of include/tnmld.h is exposed under the same name.  The
library must have been built (``__graft_entry__.build()`` or
``python paper_2605_17230_amd/build.py``); nothing here falls back to another
implementation when it is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtnmld.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tnmld.h")

TN_OK, TN_EINVAL, TN_ENOMEM, TN_EDEVICE, TN_EUNSUPPORTED, TN_ENUMERIC = 0, -1, -2, -3, -4, -5
TN_FP64, TN_FP32, TN_BF16, TN_FP32_PLAIN, TN_BF16_F64 = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": TN_FP64, "fp32": TN_FP32, "bf16": TN_BF16, "fp32plain": TN_FP32_PLAIN, "bf16f64": TN_BF16_F64}
TN_MAX_SEGMENTS = 16
TN_MAX_ROUNDS = 2


class Segment(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("chi", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n_models", ctypes.c_int32), ("rates", ctypes.c_void_p), ("model_index", ctypes.c_void_p),
        ("syndromes", ctypes.c_void_p), ("count", ctypes.c_int64), ("out_logz", ctypes.c_void_p),
        ("out_logp", ctypes.c_void_p), ("out_class", ctypes.c_void_p),
        ("rounds", ctypes.c_int32), ("reserved", ctypes.c_int32), ("meas_rates", ctypes.c_void_p),
    ]


class TNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tnmld error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtnmld.so is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, SZ, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
        seg_p = ctypes.POINTER(Segment)
        L.tn_workspace_size.restype = SZ
        L.tn_workspace_size.argtypes = [seg_p, I32, I32]
        L.tn_coset_loglik.restype = ctypes.c_int
        L.tn_coset_loglik.argtypes = [seg_p, I32, P, SZ, P]
        L.tn_decode_batch.restype = ctypes.c_int
        L.tn_decode_batch.argtypes = [seg_p, I32, D, P, SZ, P]
        L.tn_coset_loglik_backward.restype = ctypes.c_int
        L.tn_coset_loglik_backward.argtypes = [seg_p, I32, ctypes.POINTER(P), ctypes.POINTER(P), I32, P, SZ, P]
        L.tn_code_stabilizers.restype = ctypes.c_int
        L.tn_code_stabilizers.argtypes = [I32, P, P]
        L.tn_plan_info.restype = ctypes.c_int
        L.tn_plan_info.argtypes = [I32, I32, I32, ctypes.POINTER(D)]
        L.tn_plan_info_rounds.restype = ctypes.c_int
        L.tn_plan_info_rounds.argtypes = [I32, I32, I32, I32, ctypes.POINTER(D)]
        L.tn_plan_gemm_flops.restype = ctypes.c_int
        L.tn_plan_gemm_flops.argtypes = [I32, I32, I32, ctypes.POINTER(D)]
        L.tn_states_size.restype = SZ
        L.tn_states_size.argtypes = [seg_p, I32]
        L.tn_coset_loglik_save.restype = ctypes.c_int
        L.tn_coset_loglik_save.argtypes = [seg_p, I32, P, SZ, P, SZ, P]
        L.tn_coset_loglik_backward_saved.restype = ctypes.c_int
        L.tn_coset_loglik_backward_saved.argtypes = [seg_p, I32, ctypes.POINTER(P), ctypes.POINTER(P), P, SZ, P, SZ, P]
        L.tn_plan_adjoint_flops.restype = ctypes.c_int
        L.tn_plan_adjoint_flops.argtypes = [I32, I32, I32, ctypes.POINTER(D)]
        L.tn_set_tuning.restype = ctypes.c_int
        L.tn_set_tuning.argtypes = [I32, I32, I32, I32, I32]
        L.tn_set_tuning_ex.restype = ctypes.c_int
        L.tn_set_tuning_ex.argtypes = [I32, I32, I32, I32, I32, I32]
        L.tn_get_launch.restype = ctypes.c_int
        L.tn_get_launch.argtypes = [I32, I32, I32, ctypes.POINTER(I32)]
        L.tn_get_launches.restype = ctypes.c_int
        L.tn_get_launches.argtypes = [seg_p, I32, ctypes.POINTER(I32), I32, ctypes.POINTER(I32)]
        L.tn_decode_batch_noalloc.restype = ctypes.c_int
        L.tn_decode_batch_noalloc.argtypes = [seg_p, I32, D, P]
        L.tn_bitflip_workspace_size.restype = SZ
        L.tn_bitflip_workspace_size.argtypes = [seg_p, I32]
        L.tn_bitflip_decode.restype = ctypes.c_int
        L.tn_bitflip_decode.argtypes = [seg_p, I32, D, P, SZ, P]
        L.tn_bitflip_plan_info.restype = ctypes.c_int
        L.tn_bitflip_plan_info.argtypes = [I32, ctypes.POINTER(D)]
        L.tn_workspace_status.restype = ctypes.c_int
        L.tn_workspace_status.argtypes = [P, SZ, P, ctypes.POINTER(I64)]
        L.tn_last_error.restype = ctypes.c_char_p
        L.tn_last_error.argtypes = []
        _lib = L
    return _lib


def check(rc):
    if rc != TN_OK:
        raise TNError(rc, lib().tn_last_error().decode())
    return rc


def header_functions():
    """Function names declared in include/tnmld.h."""
    import re
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:size_t|int|const char\*)\s+(tn_\w+)\s*\(", src, re.M)))
