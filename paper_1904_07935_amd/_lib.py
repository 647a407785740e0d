"""ctypes binding of libplnmf.so: the names and signatures of include/nmf.h.

Argument marshalling only.  There is no fallback: if the compiled library is
missing, every call raises ``NativeLibraryMissing``.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
# PLNMF_LIB points at another build of the same library (e.g. the sanitizer build)
LIB_PATH = os.environ.get("PLNMF_LIB") or os.path.join(HERE, "libplnmf.so")

NMF_OK = 0
STATUS_NAMES = {0: "NMF_OK", -1: "NMF_E_ARG", -2: "NMF_E_SHAPE", -3: "NMF_E_WORKSPACE",
                -4: "NMF_E_HIP", -5: "NMF_E_NUMERIC", -6: "NMF_E_UNSUPPORTED", -7: "NMF_E_TIMEOUT"}
NMF_DENSE, NMF_CSR = 0, 1
NMF_FP32, NMF_BF16_PRODUCTS = 0, 1
NMF_HALF_H, NMF_HALF_W = 0, 1
NMF_FOLDIN_GIVEN, NMF_FOLDIN_WTA, NMF_FOLDIN_MLP = 0, 1, 2
NMF_MAX_K = 512
STEP_NAMES = ["gram_S", "product_R", "update_H", "product_P", "gram_Q", "update_W"]


class NativeLibraryMissing(RuntimeError):
    pass


class NmfError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


class nmf_matrix(ctypes.Structure):
    _fields_ = [("rows", c_int64), ("cols", c_int64), ("nnz", c_int64), ("format", c_int32),
                ("dense", c_void_p), ("rowptr", c_void_p), ("colidx", c_void_p),
                ("values", c_void_p)]


class nmf_info(ctypes.Structure):
    _fields_ = [("V", c_int64), ("D", c_int64), ("nnz", c_int64), ("K", c_int32),
                ("format", c_int32), ("precision", c_int32), ("tile", c_int32),
                ("w_groups", c_int32), ("h_groups", c_int32), ("sweeps_done", c_int64)]


class nmf_mlp_layout(ctypes.Structure):
    _fields_ = [("master", c_size_t), ("n_master", c_size_t), ("adam_m", c_size_t),
                ("adam_v", c_size_t), ("w1_bf16", c_size_t), ("w2_bf16", c_size_t),
                ("step", c_size_t), ("total", c_size_t)]


_P = c_void_p
SIGNATURES = {
    "nmf_workspace_bytes": [POINTER(nmf_matrix), c_int, c_int, POINTER(c_size_t)],
    "nmf_init": [POINTER(_P), POINTER(nmf_matrix), c_int, c_float, c_int, _P, _P, _P, c_size_t, _P],
    "nmf_sweep": [_P, c_int, POINTER(c_double)],
    "nmf_half": [_P, c_int],
    "nmf_mu_sweep": [_P, c_int, POINTER(c_double)],
    "nmf_objective": [_P, POINTER(c_double), POINTER(c_double)],
    "nmf_intermediates": [_P, POINTER(_P), POINTER(_P), POINTER(_P), POINTER(_P)],
    "nmf_plan_info": [_P, POINTER(nmf_info)],
    "nmf_set_stream": [_P, _P],
    "nmf_inject_status": [_P, c_int32],
    "nmf_destroy": [_P],
    "nmf_profile": [_P, c_int],
    "nmf_profile_read": [_P, POINTER(c_double), POINTER(c_int64)],
    "nmf_foldin_workspace_bytes": [_P, POINTER(nmf_matrix), c_int, POINTER(c_size_t)],
    "nmf_foldin": [_P, POINTER(nmf_matrix), _P, c_int, _P, c_int, c_int, c_double, POINTER(c_int),
                   POINTER(c_double), _P, c_size_t],
    "nmf_foldin_noalloc": [_P, POINTER(nmf_matrix), _P, c_int, _P, c_int, c_int, c_double,
                           POINTER(c_int), POINTER(c_double)],
    "nmf_mlp_param_bytes": [c_int, c_int, POINTER(nmf_mlp_layout)],
    "nmf_mlp_init": [_P, c_int, c_int, c_uint64, _P],
    "nmf_mlp_refresh": [_P, c_int, c_int, _P],
    "nmf_mlp_workspace_bytes": [c_int, c_int, c_int64, POINTER(c_size_t)],
    "nmf_mlp_predict": [_P, c_int, c_int, _P, _P, c_int64, _P, c_size_t, _P],
    "nmf_mlp_loss_grad": [_P, c_int, c_int, _P, _P, c_int64, _P, POINTER(c_double), _P, c_size_t,
                          _P],
    "nmf_mlp_adam_step": [_P, c_int, c_int, _P, c_float, _P],
    "nmf_mlp_train": [_P, c_int, c_int, _P, _P, c_int64, c_int, c_int, c_float, c_uint64, _P,
                      c_size_t, POINTER(c_double), _P],
}

_lib = None


def lib():
    """The loaded library (raises NativeLibraryMissing when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NativeLibraryMissing(
                f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        h = ctypes.CDLL(LIB_PATH)
        for name, argtypes in SIGNATURES.items():
            f = getattr(h, name)
            f.argtypes = argtypes
            f.restype = c_int
        h.nmf_last_error.argtypes = []
        h.nmf_last_error.restype = c_char_p
        _lib = h
    return _lib


def check(status):
    if status != NMF_OK:
        msg = lib().nmf_last_error()
        raise NmfError(status, msg.decode() if msg else "")
    return status


def call(name, *args):
    return check(getattr(lib(), name)(*args))
