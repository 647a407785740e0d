"""Parity of the HIP FAST-HALS path with the FP64 oracle (MI355X only).

Bars (FP32 path): relative objective within 1e-5 (relative) of the oracle's
after every sweep, and factors within 1e-3 (relative Frobenius) after 10
sweeps, from the same FP32 inputs.  Single half-steps and products are held to
tighter bounds derived from FP32 rounding of the sums involved.

Besides the Frobenius norms every factor is also checked column by column (W)
and row by row (H), and every product and Gram element by element, so that a
fault confined to one column, one tile or one group of rows cannot hide in a
norm over the whole matrix.  Per-column/row bars (calibrated on a plain FP32
NumPy transcription of Alg. 1, whose worst column sits within 2x of its
Frobenius error): W columns within 1e-3 after one half-sweep and 2e-3 after 10
sweeps; H rows within 1e-4 (one half-sweep) and 1e-3 (10 sweeps) of the RMS
row norm.  Elements of products and Grams: 1e-4 relative, above the
worst-case bound n u of an FP32 sum of n <= 1600 non-negative terms."""
import numpy as np
import pytest

import datagen
from oracle import hals
from tests.gpu_util import (EPS, col_rel_max, elem_rel_max, gpu_plan, oracle_A, oracle_run, rel_fro,
                            row_rms_max, small_bow, sparse_init)

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def _set_h(plan, H):
    """Overwrite the plan's H with the oracle's H (K x D), rounded to FP32;
    returns the rounded values in FP64 for the oracle's side."""
    import torch
    H32 = np.ascontiguousarray(np.asarray(H).T, dtype=np.float32)
    plan.Ht.copy_(torch.from_numpy(H32).to(plan.Ht.device))
    return H32.T.astype(np.float64)


@pytest.mark.parametrize("V,D,K", [(130, 97, 7), (200, 150, 16), (97, 130, 33), (300, 260, 50),
                                   (64, 64, 1), (40, 45, 40)])
def test_products_grams_and_halves_dense(cuda, V, D, K):
    A = datagen.dense_planted_uniform(V, D, max(2, K // 2), 0.01, seed=V + K)
    W0, H0 = datagen.uniform_init(V, D, K, seed=K)
    plan = gpu_plan(A, W0, H0, cuda)
    Ao = oracle_A(A)
    Wn = hals.normalize_columns(W0)
    assert rel_fro(_np(plan.W), Wn) < 1e-6
    plan.half("H")
    mid = plan.intermediates()
    H1, R, S = hals.h_half(Ao, Wn, H0, EPS)
    assert rel_fro(_np(mid["R"]), R) < 1e-5
    assert rel_fro(_np(mid["S"]), S) < 1e-5
    assert elem_rel_max(_np(mid["R"]), R) < 1e-4
    assert elem_rel_max(_np(mid["S"]), S) < 1e-4
    assert rel_fro(_np(plan.Ht).T, H1) < 1e-4
    assert row_rms_max(_np(plan.Ht).T, H1) < 1e-4
    # both W halves start from the oracle's H (rounded to FP32), so that the
    # products are compared element by element on identical inputs
    H1 = _set_h(plan, H1)
    plan.half("W")
    mid = plan.intermediates()
    W1, P, Q = hals.w_half(Ao, Wn, H1, EPS)
    assert rel_fro(_np(mid["P"]), P) < 1e-5
    assert rel_fro(_np(mid["Q"]), Q) < 1e-5
    assert elem_rel_max(_np(mid["P"]), P) < 1e-4
    assert elem_rel_max(_np(mid["Q"]), Q) < 1e-4
    # the K-step column recurrence amplifies FP32 rounding with the conditioning
    # of Q (over-parameterised K here): 5e-4 on the factor after one half-sweep
    assert rel_fro(_np(plan.W), W1) < 5e-4
    assert col_rel_max(_np(plan.W), W1) < 1e-3
    np.testing.assert_allclose(np.linalg.norm(_np(plan.W), axis=0), 1.0, rtol=1e-5)
    assert _np(plan.Ht).min() >= EPS * (1 - 1e-6)
    _, rel = plan.objective()
    _, rel_or = hals.objective(Ao, W1, H1)
    assert abs(rel - rel_or) <= 1e-5 * rel_or
    plan.close()


def test_c0_parity_50_sweeps(cuda):
    """The dense planted configuration: 1000 x 800, K = 16, 50 sweeps."""
    A = datagen.c0()
    W0, H0 = datagen.uniform_init(1000, 800, 16, seed=1)
    plan = gpu_plan(A, W0, H0, cuda)
    rel_gpu = []
    for i in range(50):
        rel_gpu += plan.sweep(1, objective=True)
        if i == 9:
            W10, Ht10 = _np(plan.W), _np(plan.Ht)
    rel_or, facs = oracle_run(A, W0, H0, 50)
    diffs = np.abs(np.array(rel_gpu) - np.array(rel_or)) / np.array(rel_or)
    print("C0 relative objective difference per sweep:", np.array2string(diffs, precision=2))
    # the bar: 1e-5 after every one of the 50 sweeps
    assert diffs.max() <= 1e-5, diffs
    assert rel_fro(W10, facs[9][0]) <= 1e-3
    assert rel_fro(Ht10.T, facs[9][1]) <= 1e-3
    assert col_rel_max(W10, facs[9][0]) <= 2e-3
    assert row_rms_max(Ht10.T, facs[9][1]) <= 1e-3
    # objective is non-increasing (up to FP32 rounding) and matches the anchor values
    assert np.all(np.diff(rel_gpu) <= 1e-6 * np.array(rel_gpu[1:]))
    plan.close()


@pytest.mark.parametrize("groups", [3, 8, 32])
def test_w_column_groups_match_oracle(cuda, monkeypatch, groups):
    """The W half split over several column groups (each holding a block of
    rows and exchanging one partial per column) against the oracle and the
    single-group run: only the order of the norm's partial sums differs."""
    A = datagen.c0()
    W0, H0 = datagen.uniform_init(1000, 800, 40, seed=3)
    base = gpu_plan(A, W0, H0, cuda)
    assert base.info()["w_groups"] == 1
    monkeypatch.setenv("NMF_W_COLUMN_GROUPS", str(groups))
    plan = gpu_plan(A, W0, H0, cuda)
    assert plan.info()["w_groups"] == groups
    r1 = np.array(base.sweep(10, objective=True))
    rg = np.array(plan.sweep(10, objective=True))
    rel_or, facs = oracle_run(A, W0, H0, 10)
    assert np.max(np.abs(rg - rel_or) / rel_or) <= 1e-5
    assert np.max(np.abs(rg - r1) / r1) <= 1e-5
    assert rel_fro(_np(plan.W), facs[-1][0]) <= 1e-3
    assert col_rel_max(_np(plan.W), facs[-1][0]) <= 2e-3
    assert row_rms_max(_np(plan.Ht).T, facs[-1][1]) <= 1e-3
    assert rel_fro(_np(plan.W), _np(base.W)) <= 1e-4
    assert col_rel_max(_np(plan.W), _np(base.W)) <= 2e-4
    np.testing.assert_allclose(np.linalg.norm(_np(plan.W), axis=0), 1.0, rtol=1e-5)
    base.close()
    plan.close()


def test_w_column_groups_across_xcds_match_oracle(cuda, monkeypatch):
    """Enough column groups that they cannot share one XCD: the W half takes
    the device-scope exchange instead of the XCD-local one; results stay within
    the bars of the oracle."""
    c = small_bow()
    K = 24
    W0, H0 = sparse_init(c, K)
    monkeypatch.setenv("NMF_W_COLUMN_GROUPS", "60")
    plan = gpu_plan(c.A, W0, H0, cuda)
    assert plan.info()["w_groups"] > 36
    rel_gpu = np.array(plan.sweep(10, objective=True))
    rel_or, facs = oracle_run(c.A, W0, H0, 10)
    assert np.max(np.abs(rel_gpu - rel_or) / rel_or) <= 1e-5
    assert rel_fro(_np(plan.W), facs[-1][0]) <= 1e-3
    assert col_rel_max(_np(plan.W), facs[-1][0]) <= 2e-3
    assert row_rms_max(_np(plan.Ht).T, facs[-1][1]) <= 1e-3
    np.testing.assert_allclose(np.linalg.norm(_np(plan.W), axis=0), 1.0, rtol=1e-5)
    plan.close()


@pytest.mark.parametrize("V, groups, K", [(40000, 32, 48), (60000, 34, 48), (150000, 84, 48),
                                           (229376, 128, 48), (150000, 84, 256)])
def test_w_half_four_rows_per_thread_matches_oracle(cuda, V, groups, K):
    """Corpora large enough that a column group holds more than two rows per
    thread (the four-row variant of the W kernel): 32 column groups on one XCD
    (the XCD-local exchange), 34 groups, more than one XCD holds (the
    device-scope exchange), 84 and 128 groups, more than one slot per polling
    lane (128 x 1792 rows is the kernel's largest V; there each product group
    serves one column group and parks only part of its row blocks in LDS
    before its wait), and 84 groups at K = 256, where the tile panel leaves
    room to park three of four blocks.  One W half against the oracle's."""
    c = datagen.bag_of_words(V, 6000 if K < 100 else 2000, 1.1, 77.0, 7)
    W0, H0 = sparse_init(c, K)
    plan = gpu_plan(c.A, W0, H0, cuda)
    assert plan.info()["w_groups"] == groups
    plan.half("W")
    Wo, _, _ = hals.w_half(oracle_A(c.A), hals.normalize_columns(W0), np.asarray(H0, np.float64), EPS)
    got = _np(plan.W)
    assert rel_fro(got, Wo) <= 5e-4
    assert col_rel_max(got, Wo) <= 1e-3
    np.testing.assert_allclose(np.linalg.norm(got, axis=0), 1.0, rtol=1e-5)
    plan.close()


def test_w_kernel_rejects_more_rows_than_it_holds(cuda):
    """V beyond what the W kernel holds (128 column groups of 1792 rows):
    nmf_init refuses the plan with NMF_E_UNSUPPORTED instead of launching a W
    update that cannot hold it."""
    from paper_1904_07935_amd._lib import NmfError
    c = datagen.bag_of_words(229377, 2000, 1.1, 77.0, 9)
    W0, H0 = sparse_init(c, 8)
    with pytest.raises(NmfError) as e:
        gpu_plan(c.A, W0, H0, cuda)
    assert e.value.status == -6


@pytest.mark.parametrize("K", [5, 24, 64])
def test_sparse_parity(cuda, K):
    c = small_bow()
    W0, H0 = sparse_init(c, K)
    plan = gpu_plan(c.A, W0, H0, cuda)
    rel_gpu = plan.sweep(10, objective=True)
    rel_or, facs = oracle_run(c.A, W0, H0, 10)
    diffs = np.abs(np.array(rel_gpu) - np.array(rel_or)) / np.array(rel_or)
    assert diffs.max() <= 1e-5, diffs
    assert rel_fro(_np(plan.W), facs[-1][0]) <= 1e-3
    assert rel_fro(_np(plan.Ht).T, facs[-1][1]) <= 1e-3
    assert col_rel_max(_np(plan.W), facs[-1][0]) <= 2e-3
    assert row_rms_max(_np(plan.Ht).T, facs[-1][1]) <= 1e-3
    plan.close()


@pytest.mark.parametrize("K", [12, 150, 200, 300, 302, 400])
def test_sparse_products_with_empty_rows_and_columns(cuda, K):
    """CSR with empty rows (terms never used) and empty columns (documents with
    no terms) and one long row spanning many nnz chunks.  K covers the narrow
    (several nonzeros per wave step) and the wide (one nonzero per step,
    prefetched item) product kernels, with and without 16-byte rows, and
    (K > 256) R formed in two column slices of W, one of them of a width that
    is not a multiple of four at K = 302."""
    rng = np.random.default_rng(5)
    V, D = 700, 500
    dense = (rng.random((V, D)) < 0.02) * rng.random((V, D))
    dense[3, :] = rng.random(D) + 0.1  # one long row (crosses chunk boundaries)
    dense[::7, :] = 0.0          # empty rows
    dense[:, ::11] = 0.0         # empty columns
    import scipy.sparse as sp
    m = sp.csr_matrix(dense.astype(np.float32))
    A = datagen.Csr(V, D, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float32))
    W0, H0 = datagen.uniform_init(V, D, K, seed=1)
    plan = gpu_plan(A, W0, H0, cuda)
    Wn = hals.normalize_columns(W0)
    Ao = oracle_A(A)
    plan.half("H")
    mid = plan.intermediates()
    H1, R, S = hals.h_half(Ao, Wn, H0, EPS)
    assert rel_fro(_np(mid["R"]), R) < 1e-5
    assert elem_rel_max(_np(mid["R"]), R) < 1e-4
    assert np.all(_np(mid["R"])[::11] == 0.0)
    H1 = _set_h(plan, H1)
    plan.half("W")
    mid = plan.intermediates()
    _, P, _ = hals.w_half(Ao, Wn, H1, EPS)
    assert rel_fro(_np(mid["P"]), P) < 1e-5
    assert elem_rel_max(_np(mid["P"]), P) < 1e-4
    assert np.all(_np(mid["P"])[::7] == 0.0)
    plan.close()


def test_objective_matches_oracle(cuda):
    A = datagen.dense_planted_uniform(300, 200, 8, 0.01, seed=3)
    W0, H0 = datagen.uniform_init(300, 200, 8, seed=1)
    plan = gpu_plan(A, W0, H0, cuda)
    f, rel = plan.objective()
    fo, relo = hals.objective(oracle_A(A), hals.normalize_columns(W0), H0.astype(np.float64))
    assert abs(rel - relo) <= 1e-6 * relo and abs(f - fo) <= 2e-6 * fo
    c = small_bow(1500, 700)
    W0, H0 = sparse_init(c, 10)
    plan2 = gpu_plan(c.A, W0, H0, cuda)
    f, rel = plan2.objective()
    fo, relo = hals.objective(oracle_A(c.A), hals.normalize_columns(W0), H0.astype(np.float64))
    assert abs(rel - relo) <= 1e-5 * relo
    plan.close()
    plan2.close()


def test_bitwise_deterministic_and_resumable(cuda):
    import torch
    c = small_bow(2000, 900)
    W0, H0 = sparse_init(c, 20)
    p1 = gpu_plan(c.A, W0, H0, cuda)
    p2 = gpu_plan(c.A, W0, H0, cuda)
    p1.sweep(6)
    p2.sweep(3)
    Ws, Hs = p2.W.clone(), p2.Ht.clone()
    p2.sweep(3)
    assert torch.equal(p1.W, p2.W) and torch.equal(p1.Ht, p2.Ht)
    p2.W.copy_(Ws)
    p2.Ht.copy_(Hs)
    p2.sweep(3)  # continue from the saved state
    assert torch.equal(p1.W, p2.W) and torch.equal(p1.Ht, p2.Ht)
    p1.close()
    p2.close()


def test_dead_column_becomes_uniform(cuda):
    """A W column whose update is <= eps in every row becomes 1/sqrt(V)."""
    V, D, K = 64, 48, 3
    rng = np.random.default_rng(0)
    A = np.zeros((V, D), dtype=np.float32)
    A[:, :] = rng.random((V, D)).astype(np.float32) * 0.1
    W0 = rng.random((V, K)).astype(np.float32)
    H0 = rng.random((K, D)).astype(np.float32)
    H0[1, :] = 50.0  # row 1 of H far too large: column 1 of W clips everywhere
    plan = gpu_plan(A, W0, H0, cuda)
    # run only the W half on the given H
    plan.half("W")
    Wo, _, _ = hals.w_half(A.astype(np.float64), hals.normalize_columns(W0), H0.astype(np.float64), EPS)
    got = _np(plan.W)
    assert rel_fro(got, Wo) < 1e-4
    assert col_rel_max(got, Wo) < 1e-3
    np.testing.assert_allclose(got[:, 1], 1.0 / np.sqrt(V), rtol=1e-6)
    plan.close()


def test_input_validation_on_device(cuda):
    import torch

    from paper_1904_07935_amd._lib import NmfError
    from paper_1904_07935_amd.api import Matrix, Plan
    V, D, K = 50, 40, 4
    W = torch.rand(V, K, device=cuda)
    Ht = torch.rand(D, K, device=cuda)
    A = torch.rand(V, D, device=cuda)
    A[3, 4] = -1.0
    with pytest.raises(NmfError) as e:
        Plan(Matrix(V, D, dense=A), W, Ht)
    assert e.value.status == -5
    A[3, 4] = 1.0
    W[0, 0] = float("nan")
    with pytest.raises(NmfError) as e:
        Plan(Matrix(V, D, dense=A), W.clone(), Ht)
    assert e.value.status == -5
    # unsorted CSR columns
    rp = torch.tensor([0, 2, 3], dtype=torch.int32, device=cuda)
    cl = torch.tensor([3, 1, 0], dtype=torch.int32, device=cuda)
    vl = torch.ones(3, device=cuda)
    with pytest.raises(NmfError) as e:
        Plan(Matrix(2, 5, rowptr=rp, col=cl, val=vl), torch.rand(2, 1, device=cuda),
             torch.rand(5, 1, device=cuda))
    assert e.value.status == -2
    # a duplicate column in a row longer than one wave step, a column out of
    # range, a negative value, and end pointers that disagree with nnz
    n = 150
    cols = list(range(n))
    cols[100] = cols[99]
    cases = [  # (row pointers, columns, values, D, expected status)
        ([0, n, n], cols, [1.0] * n, n + 1, -2),
        ([0, 2, 3], [0, 5, 1], [1.0] * 3, 5, -2),
        ([0, 2, 3], [0, 1, 2], [1.0, -1.0, 1.0], 4, -5),
        ([0, 2, 2], [0, 1, 2], [1.0] * 3, 4, -2),
    ]
    for rows_ptr, cols_, vals, Dm, code in cases:
        rp = torch.tensor(rows_ptr, dtype=torch.int32, device=cuda)
        cl = torch.tensor(cols_, dtype=torch.int32, device=cuda)
        vl = torch.tensor(vals, dtype=torch.float32, device=cuda)
        with pytest.raises(NmfError) as e:
            Plan(Matrix(2, Dm, rowptr=rp, col=cl, val=vl), torch.rand(2, 1, device=cuda),
                 torch.rand(Dm, 1, device=cuda))
        assert e.value.status == code, (rows_ptr, code, e.value.status)


def test_zero_norm_column_is_rejected(cuda):
    """A W column that is all zeros cannot be normalised: nmf_init refuses it."""
    import torch

    from paper_1904_07935_amd._lib import NmfError
    from paper_1904_07935_amd.api import Matrix, Plan
    V, D, K = 50, 40, 4
    A = torch.rand(V, D, device=cuda)
    W = torch.rand(V, K, device=cuda)
    W[:, 2] = 0.0
    with pytest.raises(NmfError) as e:
        Plan(Matrix(V, D, dense=A), W, torch.rand(D, K, device=cuda))
    assert e.value.status == -5
    assert torch.all(W[:, 2] == 0.0)


def test_timeout_reported_by_sweep_without_objective(cuda):
    """A device-side timeout of the W update (forced from the host: the status
    bit a timed-out wait sets, which makes every bounded wait give up at once)
    is reported by nmf_sweep with no objective requested, and poisons the plan."""
    from paper_1904_07935_amd._lib import NmfError
    c = small_bow(2000, 900)
    W0, H0 = sparse_init(c, 20)
    plan = gpu_plan(c.A, W0, H0, cuda)
    assert plan.info()["w_groups"] >= 2
    plan.sweep(1)  # healthy
    plan.inject_status(256)
    with pytest.raises(NmfError) as e:
        plan.sweep(1)
    assert e.value.status == -7
    with pytest.raises(NmfError) as e:
        plan.objective()
    assert e.value.status == -7
    plan.close()
    # a nmf_half timeout surfaces at the next sweep call
    plan = gpu_plan(c.A, W0, H0, cuda)
    plan.inject_status(256)
    plan.half("H")
    plan.half("W")
    with pytest.raises(NmfError) as e:
        plan.sweep(0)
    assert e.value.status == -7
    plan.close()


@pytest.mark.parametrize("K", [16, 200])
def test_dense_rows_in_p_product(cuda, monkeypatch, K):
    """The densest rows of A (the Zipf head) multiplied as a dense block on the
    matrix cores -- scattered into P, and added into R from the rows of W they
    name -- the rest by the sparse products (NMF_DENSE_ROWS=1 forces it at
    this size): R and P element by element and ten sweeps' objectives against
    the oracle."""
    monkeypatch.setenv("NMF_DENSE_ROWS", "1")
    c = small_bow()
    lens = np.diff(c.A.rowptr)
    assert np.sum((lens > 128) & (16 * lens >= c.A.cols)) >= 3  # several rows qualify
    W0, H0 = sparse_init(c, K)
    plan = gpu_plan(c.A, W0, H0, cuda)
    Ao = oracle_A(c.A)
    plan.half("H")  # R = A^T W: the dense rows' share added by the matrix cores
    R = np.asarray(Ao.T @ hals.normalize_columns(W0))
    assert elem_rel_max(_np(plan.intermediates()["R"]), R) < 1e-4
    plan.close()
    plan = gpu_plan(c.A, W0, H0, cuda)
    plan.half("W")
    P = np.asarray(Ao @ H0.astype(np.float32).astype(np.float64).T)
    assert elem_rel_max(_np(plan.intermediates()["P"]), P) < 1e-4
    plan.close()
    plan = gpu_plan(c.A, W0, H0, cuda)
    rel = np.array(plan.sweep(10, objective=True))
    rel_or, _ = oracle_run(c.A, W0, H0, 10)
    assert np.max(np.abs(rel - rel_or) / np.array(rel_or)) <= 1e-5
    plan.close()
