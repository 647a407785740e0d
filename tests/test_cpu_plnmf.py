"""PL-NMF-cpu (the FP64 OpenMP host baseline, libplnmf_cpu.so) against the
FP64 oracle: both compute Alg. 1 in FP64, so they agree to rounding (1e-10
relative on the objective and the factors) for every tile width, including
ragged last tiles, dense and sparse A, and any thread count (the reductions
use fixed chunks, so the result is the same bit for bit)."""
import numpy as np
import pytest

import datagen
from oracle import hals
from tests.gpu_util import oracle_A, rel_fro


def _oracle(A, W0, H0, n):
    Ao = oracle_A(A)
    W, H = hals.normalize_columns(W0), H0.astype(np.float64)
    rels = []
    for _ in range(n):
        W, H = hals.sweep(Ao, W, H, 1e-16)
        rels.append(hals.objective(Ao, W, H)[1])
    return np.array(rels), W, H


@pytest.fixture(scope="module")
def cpu():
    from paper_1904_07935_amd import cpu
    try:
        cpu.lib()
    except RuntimeError:
        pytest.skip("libplnmf_cpu.so not built")
    return cpu


@pytest.mark.parametrize("tile", [0, 1, 3, 7, 40])
def test_dense_matches_oracle(cpu, tile):
    A = datagen.dense_planted_uniform(120, 90, 8, 0.01, seed=2)
    W0, H0 = datagen.uniform_init(120, 90, 40, seed=1)
    p = cpu.CpuPlan(A, W0, H0, tile=tile, threads=4)
    rel = np.array(p.sweep(5, objective=True))
    ref, Wo, Ho = _oracle(A, W0, H0, 5)
    assert np.max(np.abs(rel - ref) / ref) <= 1e-10
    assert rel_fro(p.W, Wo) <= 1e-10 and rel_fro(p.Ht.T, Ho) <= 1e-10


@pytest.mark.parametrize("K,tile", [(24, 0), (24, 5), (50, 32)])
def test_sparse_matches_oracle(cpu, K, tile):
    c = datagen.bag_of_words(1500, 700, 1.1, 40.0, 3)
    W0, H0 = datagen.uniform_init_matched(1500, 700, K, datagen.mean_value(c.A), 1)
    p = cpu.CpuPlan(c.A, W0, H0, tile=tile, threads=3)
    rel = np.array(p.sweep(6, objective=True))
    ref, Wo, Ho = _oracle(c.A, W0, H0, 6)
    assert np.max(np.abs(rel - ref) / ref) <= 1e-10
    assert rel_fro(p.W, Wo) <= 1e-10 and rel_fro(p.Ht.T, Ho) <= 1e-10


def test_thread_count_does_not_change_the_result(cpu):
    c = datagen.bag_of_words(900, 500, 1.1, 30.0, 4)
    W0, H0 = datagen.uniform_init_matched(900, 500, 20, datagen.mean_value(c.A), 1)
    outs = []
    for th in (1, 2, 5):
        p = cpu.CpuPlan(c.A, W0, H0, threads=th)
        p.sweep(3)
        outs.append((p.W.copy(), p.Ht.copy()))
    for W, H in outs[1:]:
        assert np.array_equal(W, outs[0][0]) and np.array_equal(H, outs[0][1])


def test_default_tile_is_the_sec5_choice(cpu):
    A = datagen.dense_planted_uniform(500, 450, 8, 0.01, seed=2)
    W0, H0 = datagen.uniform_init(500, 450, 400, seed=1)
    assert cpu.CpuPlan(A, W0, H0).info()["tile"] == 20  # round(sqrt(400))


def test_library_exports_every_declared_symbol(cpu):
    import ctypes
    import os
    import re
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                       "nmf_cpu.h")
    names = re.findall(r"^int\s+(nmf_cpu_\w+)\s*\(", open(hdr).read(), re.M)
    assert len(names) == 4
    h = ctypes.CDLL(cpu.LIB_PATH)
    for n in names:
        assert hasattr(h, n), n


def test_bad_arguments_are_rejected(cpu):
    from ctypes import byref, c_void_p
    h = c_void_p()
    W = np.ones((4, 2))
    Ht = np.ones((3, 2))
    A = np.ones((4, 3), np.float32)
    L = cpu.lib()
    ptr = cpu._ptr
    from ctypes import c_double, c_float
    assert L.nmf_cpu_init(byref(h), 4, 3, None, None, ptr(A, c_float), 5, 1e-16, 0, 1,
                          ptr(W, c_double), ptr(Ht, c_double)) == -2          # K > min(V, D)
    assert L.nmf_cpu_init(byref(h), 4, 3, None, None, ptr(A, c_float), 2, 0.0, 0, 1,
                          ptr(W, c_double), ptr(Ht, c_double)) == -1          # eps
    A[1, 1] = -1.0
    assert L.nmf_cpu_init(byref(h), 4, 3, None, None, ptr(A, c_float), 2, 1e-16, 0, 1,
                          ptr(W, c_double), ptr(Ht, c_double)) == -5          # negative entry
