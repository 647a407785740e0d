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


@pytest.mark.parametrize("K", [40, 200])
def test_kernel_change_within_one_plan(cuda, monkeypatch, K):
    """The two kernels read the Gram's panels in different orders; a plan whose
    kernel choice changes between H halves (NMF_H_KERNEL) clears the other
    order's entries first.  Three halves, rows -> lds -> rows, each against the
    oracle's H half from the previous result."""
    V, D = 300, 1000
    A = datagen.dense_planted_uniform(V, D, K // 2, 0.01, seed=D + K + 1)
    W0, H0 = datagen.uniform_init(V, D, K, seed=K + 3)
    Ao = oracle_A(A)
    Wn = hals.normalize_columns(W0)
    plan = gpu_plan(A, W0, H0, cuda)
    H = H0.astype(np.float64)
    for kern in ("rows", "lds", "rows"):
        monkeypatch.setenv("NMF_H_KERNEL", kern)
        plan.half("H")
        H, _, _ = hals.h_half(Ao, Wn, H, EPS)
        got = _np(plan.Ht).T
        assert rel_fro(got, H) < 1e-4, kern
        assert row_rms_max(got, H) < 2e-4, kern
        H = got.astype(np.float64)  # the next half starts where the GPU is
    plan.close()


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


@pytest.mark.parametrize("V,D,K", [(300, 1000, 40), (400, 900, 160), (700, 700, 400)])
@pytest.mark.parametrize("tile", [16, 64])
def test_tile_widths_match_oracle(cuda, monkeypatch, V, D, K, tile):
    """NMF_TILE_T: the H update with 16- or 64-column tiles (the tile-size
    study's kernels) against the untiled oracle -- the tiling only reorders
    the sums (Alg. 2).  A width whose double-buffered panel does not fit the
    LDS (64 at K = 400) falls back to 32, reported by the plan."""
    monkeypatch.setenv("NMF_TILE_T", str(tile))
    A = datagen.dense_planted_uniform(V, D, max(2, K // 2), 0.01, seed=D + K)
    W0, H0 = datagen.uniform_init(V, D, K, seed=K + 1)
    Ao = oracle_A(A)
    H1, _, _ = hals.h_half(Ao, hals.normalize_columns(W0), H0, EPS)
    plan = gpu_plan(A, W0, H0, cuda)
    want = tile if (tile == 16 or K <= 160) else 32
    assert plan.info()["tile"] == want
    plan.half("H")
    got = _np(plan.Ht).T
    assert rel_fro(got, H1) < 1e-4
    assert row_rms_max(got, H1) < 2e-4
    rel = np.array(plan.sweep(3, objective=True))
    assert np.all(np.isfinite(rel))
    plan.close()


def test_tile_width_in_foldin(cuda, monkeypatch):
    """Fold-in (the H update with W fixed) at 16-column tiles against the oracle."""
    import torch

    from paper_1904_07935_amd.api import Matrix
    monkeypatch.setenv("NMF_TILE_T", "16")
    c = datagen.bag_of_words(2000, 900, 1.1, 77.0, 2)
    K = 48
    W0, H0 = datagen.uniform_init_matched(2000, 900, K, datagen.mean_value(c.A), 1)
    plan = gpu_plan(c.A, W0, H0, cuda)
    assert plan.info()["tile"] == 16
    W = _np(plan.W)
    new = datagen.bag_of_words_docs(500, 1.1, 77.0, 7, c.perm, c.idf)
    _, Hn = datagen.uniform_init_matched(2000, 500, K, datagen.mean_value(new), 4)
    Ht = torch.tensor(np.ascontiguousarray(Hn.T), device=cuda)
    trace = plan.foldin(Matrix.from_csr(new, cuda), Ht, init="given", n_sweeps=10)
    from tests.gpu_util import rows_csr_to_oracle
    An = rows_csr_to_oracle(new)
    rels = [hals.objective(An, W, Hn.astype(np.float64))[1]]
    hals.foldin(An, W, Hn, EPS, 10, on_sweep=lambda i, H: rels.append(hals.objective(An, W, H)[1]))
    d = np.abs(np.array(trace) - np.array(rels)) / np.array(rels)
    assert d.max() <= 1e-5
    plan.close()
