"""Shared helpers of the GPU parity tests: run the HIP path and the FP64 oracle
from the same seeded FP32 inputs."""
import numpy as np
import scipy.sparse as sp

import datagen
from oracle import hals

EPS = 1e-16


def rel_fro(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def col_rel_max(x, ref):
    """Largest relative L2 error over the columns: max_k ||x_k - r_k|| / ||r_k||.
    For W (unit-norm columns) this catches one bad column that a Frobenius norm
    over all K columns would dilute by sqrt(K)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.linalg.norm(x - ref, axis=0) / np.linalg.norm(ref, axis=0)))


def row_rms_max(x, ref):
    """Largest L2 error over the rows, relative to the RMS row norm of ref:
    max_k ||x_k - r_k|| / sqrt(mean_k ||r_k||^2).  For H (rows of very
    different norms, some clipped to eps) a per-row relative error would be
    dominated by near-zero rows; this scale still flags one bad row."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.sqrt(np.mean(np.sum(ref * ref, axis=1)))
    return float(np.max(np.linalg.norm(x - ref, axis=1)) / scale)


def elem_rel_max(x, ref, floor=1e-6):
    """Largest element-wise relative error, |x - r| / max(|r|, floor * max|r|).
    The products and Grams of non-negative factors have non-negative entries
    whose FP32 sums carry a relative error of a few units of rounding times
    the square root of the number of terms."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.maximum(np.abs(ref), floor * np.max(np.abs(ref)))
    return float(np.max(np.abs(x - ref) / den))


def gpu_plan(A, W0, H0, dev, precision="fp32", eps=EPS):
    """A: dense float32 ndarray or datagen.Csr (V rows).  H0 is K x D."""
    import torch

    from paper_1904_07935_amd.api import Matrix, Plan

    M = Matrix.from_csr(A, dev) if isinstance(A, datagen.Csr) else Matrix.from_dense(A, dev)
    W = torch.tensor(np.ascontiguousarray(W0, dtype=np.float32), device=dev)
    Ht = torch.tensor(np.ascontiguousarray(H0.T, dtype=np.float32), device=dev)
    return Plan(M, W, Ht, eps=eps, precision=precision)


def oracle_A(A):
    if isinstance(A, datagen.Csr):
        return sp.csr_matrix((A.val.astype(np.float64), A.col, A.rowptr), shape=(A.rows, A.cols))
    return np.asarray(A, dtype=np.float64)


def oracle_run(A, W0, H0, sweeps, eps=EPS):
    """Per-sweep relative objectives and the factors after each sweep."""
    Ao = oracle_A(A)
    W = hals.normalize_columns(W0)
    H = np.asarray(H0, dtype=np.float64)
    rels, facs = [], []
    for _ in range(sweeps):
        W, H = hals.sweep(Ao, W, H, eps)
        rels.append(hals.objective(Ao, W, H)[1])
        facs.append((W.copy(), H.copy()))
    return rels, facs


def small_bow(V=3000, D=1200, seed=2):
    return datagen.bag_of_words(V, D, 1.1, 77.0, seed)


def sparse_init(c, K, seed=1):
    """Scale-matched U[0,1) init for a bag-of-words corpus (see datagen)."""
    return datagen.uniform_init_matched(c.A.rows, c.A.cols, K, datagen.mean_value(c.A), seed)


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float64."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def rows_csr_to_oracle(csr):
    """A doc-major CSR (rows = documents) as the oracle's V x D' matrix."""
    m = sp.csr_matrix((csr.val.astype(np.float64), csr.col, csr.rowptr), shape=(csr.rows, csr.cols))
    return m.T.tocsr()
