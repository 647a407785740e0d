"""The two H-update kernels against the oracle (MI355X only).

The library picks the rows-in-registers kernel (four waves of 32 rows per
workgroup, rows in VGPRs, phase 2 split over lane pairs) for many rows and the
LDS-resident kernel (32 rows per workgroup) otherwise; NMF_H_KERNEL forces
either.  Both run here on every shape: ragged last tiles (K not a multiple of
32), a partly filled last workgroup (waves with no rows at all), one tile
(K <= 32), and K = 512 (16 tiles, the largest rank)."""
import numpy as np
import pytest

import datagen
from oracle import hals
from tests.gpu_util import EPS, gpu_plan, oracle_A, rel_fro, row_rms_max

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("V,D,K", [(300, 1000, 40), (120, 300, 7), (600, 5000, 200),
                                   (700, 700, 416), (600, 600, 512), (90, 33, 32)])
def test_h_half_both_kernels_match_oracle(cuda, monkeypatch, V, D, K):
    A = datagen.dense_planted_uniform(V, D, max(2, K // 2), 0.01, seed=D + K)
    W0, H0 = datagen.uniform_init(V, D, K, seed=K + 1)
    Ao = oracle_A(A)
    H1, _, _ = hals.h_half(Ao, hals.normalize_columns(W0), H0, EPS)
    got = {}
    for kern in ("rows", "lds"):
        monkeypatch.setenv("NMF_H_KERNEL", kern)
        plan = gpu_plan(A, W0, H0, cuda)
        plan.half("H")
        got[kern] = _np(plan.Ht).T
        plan.close()
        assert rel_fro(got[kern], H1) < 1e-4, kern
        assert row_rms_max(got[kern], H1) < 2e-4, kern
        assert got[kern].min() >= EPS * (1 - 1e-6)
    # the two kernels differ only in the summation order of the tile product
    assert rel_fro(got["rows"], got["lds"]) < 1e-4


def test_rows_kernel_full_sweeps_match_oracle(cuda, monkeypatch):
    """Ten sweeps of a sparse corpus with the rows kernel forced: the per-sweep
    objective bar of the FP32 path."""
    monkeypatch.setenv("NMF_H_KERNEL", "rows")
    c = datagen.bag_of_words(3000, 1500, 1.1, 77.0, 2)
    K = 48
    W0, H0 = datagen.uniform_init_matched(3000, 1500, K, datagen.mean_value(c.A), 1)
    plan = gpu_plan(c.A, W0, H0, cuda)
    rel = np.array(plan.sweep(10, objective=True))
    plan.close()
    Ao = oracle_A(c.A)
    W, H = hals.normalize_columns(W0), H0.astype(np.float64)
    ref = []
    for _ in range(10):
        W, H = hals.sweep(Ao, W, H, EPS)
        ref.append(hals.objective(Ao, W, H)[1])
    ref = np.array(ref)
    assert np.max(np.abs(rel - ref) / ref) <= 1e-5
