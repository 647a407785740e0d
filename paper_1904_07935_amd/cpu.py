"""ctypes binding of libplnmf_cpu.so (include/nmf_cpu.h): PL-NMF-cpu, the
paper's tiled FAST-HALS on the host in FP64 with OpenMP.  A comparison
baseline with entry points of its own; the GPU library never calls it.
Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PLNMF_CPU_LIB") or os.path.join(HERE, "libplnmf_cpu.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (paper_1904_07935_amd.build)")
        h = ctypes.CDLL(LIB_PATH)
        h.nmf_cpu_init.argtypes = [POINTER(c_void_p), c_int64, c_int64, POINTER(c_int32),
                                   POINTER(c_int32), POINTER(c_float), c_int, c_double, c_int, c_int,
                                   POINTER(c_double), POINTER(c_double)]
        h.nmf_cpu_sweep.argtypes = [c_void_p, c_int, POINTER(c_double)]
        h.nmf_cpu_info.argtypes = [c_void_p, POINTER(c_int), POINTER(c_int)]
        h.nmf_cpu_destroy.argtypes = [c_void_p]
        for f in (h.nmf_cpu_init, h.nmf_cpu_sweep, h.nmf_cpu_info, h.nmf_cpu_destroy):
            f.restype = c_int
        _lib = h
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(POINTER(t))


class CpuPlan:
    """PL-NMF-cpu on a datagen.Csr (V rows) or a dense float32 array.  W0 [V,K]
    and H0 [K,D] are copied to FP64 (``self.W``, ``self.Ht``, updated in place)."""

    def __init__(self, A, W0, H0, eps=1e-16, tile=0, threads=0):
        self.W = np.ascontiguousarray(W0, dtype=np.float64)
        self.Ht = np.ascontiguousarray(np.asarray(H0, dtype=np.float64).T)
        V, K = self.W.shape
        D = self.Ht.shape[0]
        if hasattr(A, "rowptr"):
            self._keep = (np.ascontiguousarray(A.rowptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                          np.ascontiguousarray(A.val, np.float32))
            rp, cl, vl = _ptr(self._keep[0], c_int32), _ptr(self._keep[1], c_int32), _ptr(self._keep[2], c_float)
        else:
            self._keep = (np.ascontiguousarray(A, np.float32),)
            rp, cl, vl = None, None, _ptr(self._keep[0], c_float)
        h = c_void_p()
        rc = lib().nmf_cpu_init(byref(h), V, D, rp, cl, vl, K, eps, tile, threads,
                                _ptr(self.W, c_double), _ptr(self.Ht, c_double))
        if rc != 0:
            raise RuntimeError(f"nmf_cpu_init failed with status {rc}")
        self.h = h

    def sweep(self, n=1, objective=False):
        out = (c_double * n)() if objective else None
        rc = lib().nmf_cpu_sweep(self.h, n, out)
        if rc != 0:
            raise RuntimeError(f"nmf_cpu_sweep failed with status {rc}")
        return list(out) if objective else None

    def info(self):
        t, th = c_int(), c_int()
        lib().nmf_cpu_info(self.h, byref(t), byref(th))
        return {"tile": t.value, "threads": th.value}

    def close(self):
        if getattr(self, "h", None):
            lib().nmf_cpu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
