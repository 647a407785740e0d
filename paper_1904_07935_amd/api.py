"""Python face of the library: torch tensors in, C-ABI calls out.

Argument marshalling only -- every step runs in the library's HIP kernels.
PyTorch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_size_t, c_void_p

import numpy as np
import torch

from . import _lib as L

_ALIGN = 256


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _aligned_bytes(nbytes, device):
    """Device byte buffer whose data pointer is 256-byte aligned."""
    raw = torch.empty(int(nbytes) + _ALIGN, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % _ALIGN
    return raw, raw[off: off + int(nbytes)]


def _view(buf, ptr, count, dtype):
    """A tensor view into `buf` (uint8) at device address `ptr`."""
    off = ptr - buf.data_ptr()
    itemsize = torch.empty((), dtype=dtype).element_size()
    return buf[off: off + count * itemsize].view(dtype)


class Matrix:
    """A device matrix handed across the boundary (keeps its tensors alive)."""

    def __init__(self, rows, cols, dense=None, rowptr=None, col=None, val=None):
        self.rows, self.cols = int(rows), int(cols)
        self.dense, self.rowptr, self.col, self.val = dense, rowptr, col, val
        m = L.nmf_matrix()
        m.rows, m.cols = self.rows, self.cols
        if dense is not None:
            assert dense.dtype == torch.float32 and dense.is_contiguous()
            m.format = L.NMF_DENSE
            m.nnz = self.rows * self.cols
            m.dense = dense.data_ptr()
        else:
            assert rowptr.dtype == torch.int32 and col.dtype == torch.int32
            assert val.dtype == torch.float32
            m.format = L.NMF_CSR
            m.nnz = int(col.numel())
            m.rowptr = rowptr.data_ptr()
            m.colidx = col.data_ptr() if col.numel() else None
            m.values = val.data_ptr() if val.numel() else None
        self.c = m

    @property
    def is_sparse(self):
        return self.dense is None

    @staticmethod
    def from_dense(a, device):
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return Matrix(t.shape[0], t.shape[1], dense=t)

    @staticmethod
    def from_csr(csr, device):
        """From an object with rows, cols, rowptr, col, val (numpy arrays)."""
        rp = torch.as_tensor(np.ascontiguousarray(csr.rowptr, dtype=np.int32)).to(device)
        cl = torch.as_tensor(np.ascontiguousarray(csr.col, dtype=np.int32)).to(device)
        vl = torch.as_tensor(np.ascontiguousarray(csr.val, dtype=np.float32)).to(device)
        return Matrix(csr.rows, csr.cols, rowptr=rp, col=cl, val=vl)


PRECISIONS = {"fp32": L.NMF_FP32, "bf16": L.NMF_BF16_PRODUCTS}


class Plan:
    """FAST-HALS on one GPU: ``W`` [V,K] and ``Ht`` [D,K] are updated in place."""

    def __init__(self, A: Matrix, W: torch.Tensor, Ht: torch.Tensor, eps=1e-16, precision="fp32"):
        assert W.dtype == torch.float32 and Ht.dtype == torch.float32
        assert W.is_contiguous() and Ht.is_contiguous()
        self.A, self.W, self.Ht = A, W, Ht
        self.K = int(W.shape[1])
        self.precision = precision
        prec = PRECISIONS[precision]
        nb = c_size_t(0)
        L.call("nmf_workspace_bytes", byref(A.c), self.K, prec, byref(nb))
        self._raw, self.ws = _aligned_bytes(nb.value, W.device)
        h = c_void_p()
        L.call("nmf_init", byref(h), byref(A.c), self.K, float(eps), prec, W.data_ptr(),
               Ht.data_ptr(), self.ws.data_ptr(), nb.value, _stream())
        self.h = h
        self.eps = eps

    def _sync_stream(self):
        L.call("nmf_set_stream", self.h, _stream())

    def sweep(self, n=1, objective=False):
        self._sync_stream()
        if objective:
            out = (c_double * n)()
            L.call("nmf_sweep", self.h, n, out)
            return list(out)
        L.call("nmf_sweep", self.h, n, None)
        return None

    def mu_sweep(self, n=1, objective=False):
        """n iterations of the multiplicative-update baseline (nmf_mu_sweep)."""
        self._sync_stream()
        if objective:
            out = (c_double * n)()
            L.call("nmf_mu_sweep", self.h, n, out)
            return list(out)
        L.call("nmf_mu_sweep", self.h, n, None)
        return None

    def half(self, which):
        self._sync_stream()
        L.call("nmf_half", self.h, {"H": L.NMF_HALF_H, "W": L.NMF_HALF_W}[which])

    def objective(self):
        self._sync_stream()
        f, r = c_double(), c_double()
        L.call("nmf_objective", self.h, byref(f), byref(r))
        return f.value, r.value

    def intermediates(self):
        """Views of P [V,K], Q [K,K], R [D,K], S [K,K] inside the workspace."""
        ptrs = [c_void_p() for _ in range(4)]
        L.call("nmf_intermediates", self.h, *[byref(p) for p in ptrs])
        V, D, K = self.W.shape[0], self.Ht.shape[0], self.K
        shapes = [(V, K), (K, K), (D, K), (K, K)]
        out = {}
        for name, p, shp in zip("PQRS", ptrs, shapes):
            out[name] = _view(self.ws, p.value, shp[0] * shp[1], torch.float32).view(*shp)
        return out

    def profile(self, enable=True):
        """Record HIP events around every step (see ``profile_read``)."""
        L.call("nmf_profile", self.h, 1 if enable else 0)

    def profile_read(self):
        """{step: (total ms, launches)} since the last read; synchronises."""
        n = len(L.STEP_NAMES)
        ms = (c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        L.call("nmf_profile_read", self.h, ms, cnt)
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.STEP_NAMES)}

    def inject_status(self, bits=256):
        """Fault injection for error-path tests (NMF_STATUS_TIMEOUT)."""
        self._sync_stream()
        L.call("nmf_inject_status", self.h, int(bits))

    def info(self):
        i = L.nmf_info()
        L.call("nmf_plan_info", self.h, byref(i))
        return {f: getattr(i, f) for f, _ in L.nmf_info._fields_}

    def foldin(self, AnewT: Matrix, Ht_new: torch.Tensor, init="given", mlp=None, n_sweeps=10,
               trace=True, tol=0.0, noalloc=False):
        """H-only sweeps for new documents (rows of AnewT) with this plan's W fixed.

        ``n_sweeps`` is the most sweeps run; with ``tol > 0`` the call stops
        after the first sweep lowering the relative objective by less than tol.
        ``noalloc=True`` calls nmf_foldin_noalloc (the library's own device
        array as workspace) instead of allocating one here.
        Returns the trace (objective after the init and after each sweep run)
        or None; ``self.foldin_sweeps`` holds the number of sweeps run."""
        self._sync_stream()
        mode = {"given": L.NMF_FOLDIN_GIVEN, "wta": L.NMF_FOLDIN_WTA, "mlp": L.NMF_FOLDIN_MLP}[init]
        hidden = mlp.hidden if mlp is not None else 0
        params = mlp.blob.data_ptr() if mlp is not None else None
        tr = (c_double * (n_sweeps + 1))() if trace else None
        done = ctypes.c_int(0)
        if noalloc:
            L.call("nmf_foldin_noalloc", self.h, byref(AnewT.c), Ht_new.data_ptr(), mode, params,
                   hidden, n_sweeps, float(tol), byref(done), tr)
        else:
            nb = c_size_t(0)
            L.call("nmf_foldin_workspace_bytes", self.h, byref(AnewT.c), hidden, byref(nb))
            raw, ws = _aligned_bytes(nb.value, Ht_new.device)
            L.call("nmf_foldin", self.h, byref(AnewT.c), Ht_new.data_ptr(), mode, params, hidden,
                   n_sweeps, float(tol), byref(done), tr, ws.data_ptr(), nb.value)
            del raw
        self.foldin_sweeps = done.value
        return list(tr)[: done.value + 1] if trace else None

    def close(self):
        if getattr(self, "h", None):
            L.call("nmf_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The fold-in warm-start network: parameters in one device blob."""

    def __init__(self, K, hidden=512, device="cuda", seed=0):
        self.K, self.hidden = int(K), int(hidden)
        lay = L.nmf_mlp_layout()
        L.call("nmf_mlp_param_bytes", self.K, self.hidden, byref(lay))
        self.layout = lay
        self._raw, self.blob = _aligned_bytes(lay.total, device)
        if seed is not None:
            L.call("nmf_mlp_init", self.blob.data_ptr(), self.K, self.hidden, int(seed), _stream())
        self._ws_raw = None
        self._ws = None
        self._ws_batch = 0

    def _masters_flat(self):
        return self.blob[self.layout.master: self.layout.master + 4 * self.layout.n_master].view(torch.float32)

    def masters(self):
        f = self._masters_flat()
        K, H = self.K, self.hidden
        o = 0
        out = {}
        for name, shp in (("W1", (H, K)), ("b1", (H,)), ("W2", (K, H)), ("b2", (K,))):
            n = int(np.prod(shp))
            out[name] = f[o: o + n].view(*shp)
            o += n
        return out

    def set_masters(self, params):
        m = self.masters()
        for k, v in params.items():
            m[k].copy_(torch.as_tensor(np.asarray(v, dtype=np.float32)))
        L.call("nmf_mlp_refresh", self.blob.data_ptr(), self.K, self.hidden, _stream())

    def working_bf16(self):
        K, H = self.K, self.hidden
        w1 = self.blob[self.layout.w1_bf16: self.layout.w1_bf16 + 2 * H * K].view(torch.bfloat16).view(H, K)
        w2 = self.blob[self.layout.w2_bf16: self.layout.w2_bf16 + 2 * K * H].view(torch.bfloat16).view(K, H)
        return w1, w2

    def _workspace(self, batch):
        if self._ws is None or batch > self._ws_batch:
            nb = c_size_t(0)
            L.call("nmf_mlp_workspace_bytes", self.K, self.hidden, int(batch), byref(nb))
            self._ws_raw, self._ws = _aligned_bytes(nb.value, self.blob.device)
            self._ws_batch = batch
        return self._ws

    def forward(self, X, batch=8192):
        X = X.contiguous()
        Y = torch.empty_like(X)
        ws = self._workspace(min(batch, max(1, X.shape[0])))
        L.call("nmf_mlp_predict", self.blob.data_ptr(), self.K, self.hidden, X.data_ptr(),
               Y.data_ptr(), X.shape[0], ws.data_ptr(), ws.numel(), _stream())
        return Y

    def loss_grad(self, X, Y):
        X, Y = X.contiguous(), Y.contiguous()
        ws = self._workspace(X.shape[0])
        g = torch.empty(self.layout.n_master, dtype=torch.float32, device=X.device)
        loss = c_double()
        L.call("nmf_mlp_loss_grad", self.blob.data_ptr(), self.K, self.hidden, X.data_ptr(),
               Y.data_ptr(), X.shape[0], g.data_ptr(), byref(loss), ws.data_ptr(), ws.numel(),
               _stream())
        K, H = self.K, self.hidden
        o = 0
        grads = {}
        for name, shp in (("W1", (H, K)), ("b1", (H,)), ("W2", (K, H)), ("b2", (K,))):
            n = int(np.prod(shp))
            grads[name] = g[o: o + n].view(*shp)
            o += n
        return loss.value, grads, g

    def adam_step(self, flat_grads, lr=1e-3):
        L.call("nmf_mlp_adam_step", self.blob.data_ptr(), self.K, self.hidden,
               flat_grads.data_ptr(), float(lr), _stream())

    def train(self, X, Y, epochs=10, batch=1024, lr=1e-3, seed=0):
        X, Y = X.contiguous(), Y.contiguous()
        ws = self._workspace(batch)
        losses = (c_double * epochs)()
        L.call("nmf_mlp_train", self.blob.data_ptr(), self.K, self.hidden, X.data_ptr(),
               Y.data_ptr(), X.shape[0], int(epochs), int(batch), float(lr), int(seed),
               ws.data_ptr(), ws.numel(), losses, _stream())
        return list(losses)
