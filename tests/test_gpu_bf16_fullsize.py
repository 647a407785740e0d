"""BF16 product variant (error against the FP64 oracle stated, not bounded by
the FP32 bar) and full-size configurations (MI355X only).

Full-size parity runs the configurations at their stated sizes in the launch
configuration the benchmark times and compares with the oracle from the same
FP32 inputs: the 26,000 x 11,000 corpus for 10 sweeps at every rank, the dense
10^4 x 10^4 problem for 5 sweeps, and on the 10^5 x 3*10^5 corpus one W half
(every column against the oracle's) plus the row-independent H half on sampled
documents and properties that hold at any size."""
import numpy as np
import pytest

import datagen
from oracle import hals
from tests.gpu_util import (EPS, bf16_round, col_rel_max, elem_rel_max, gpu_plan, oracle_A, oracle_run,
                            rel_fro, row_rms_max, small_bow, sparse_init)

pytestmark = pytest.mark.gpu

BF16_REL_BOUND = 1e-2  # stated bound on |rel_bf16 - rel_fp64| / rel_fp64 at these sizes
# FP32 against the FP64 oracle on the dense image-shaped problem after sweep 1:
# a plain FP32 NumPy transcription of Alg. 1 differs by 3.9e-7, 7.8e-6, 2.2e-4,
# 2.0e-4 and 6.1e-4 after sweeps 1-5 (rows of H clipped to eps in sweep 1 revive
# at rounding level), so sweeps 2-5 are held to a bound of that order
C2_FP32_LATER_BOUND = 1e-2


def _np(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def test_bf16_products_dense_error_stated(cuda):
    """On the dense planted parity problem (where the FP32 path tracks the
    oracle sweep by sweep), the BF16-product path's error is stated and bounded."""
    A = datagen.c0()
    W0, H0 = datagen.uniform_init(1000, 800, 16, seed=1)
    rel_or, _ = oracle_run(A, W0, H0, 10)
    p32 = gpu_plan(A, W0, H0, cuda)
    p16 = gpu_plan(A, W0, H0, cuda, precision="bf16")
    r32 = np.array(p32.sweep(10, objective=True))
    r16 = np.array(p16.sweep(10, objective=True))
    e32 = np.abs(r32 - rel_or) / rel_or
    # BF16 cannot represent A better than delta = ||A - bf16(A)|| / ||A||; where
    # the achievable residual is of that size the error is bounded in absolute
    # relative-objective units by a multiple of it
    delta = rel_fro(bf16_round(A), A)
    err = np.abs(r16 - rel_or)
    print(f"bf16 |rel - rel_fp64| per sweep (delta {delta:.2e}):", np.array2string(err, precision=2))
    assert e32.max() <= 1e-5
    assert np.all(err <= 2.0 * delta + BF16_REL_BOUND * np.array(rel_or))
    assert np.all(np.isfinite(r16))
    p32.close()
    p16.close()


@pytest.mark.parametrize("K", [24, 160, 400])
def test_bf16_products_sparse_error_stated(cuda, K):
    """K = 24: several nonzeros per wave step; K = 160: the one-nonzero-per-step
    kernel with its prefetched item, gathering BF16 rows; K = 400: the same with
    one 16-byte load of eight BF16 values per lane."""
    c = small_bow()
    W0, H0 = sparse_init(c, K)
    rel_or, _ = oracle_run(c.A, W0, H0, 8)
    p16 = gpu_plan(c.A, W0, H0, cuda, precision="bf16")
    r16 = np.array(p16.sweep(8, objective=True))
    e16 = np.abs(r16 - rel_or) / rel_or
    print("bf16 sparse rel-objective error per sweep:", np.array2string(e16, precision=2))
    assert e16.max() <= BF16_REL_BOUND
    # the BF16 products themselves: R after the next H half against FP64
    p16.half("H")
    mid = p16.intermediates()
    import scipy.sparse as sp
    Ao = oracle_A(c.A)
    R = np.asarray(Ao.T @ _np(p16.W))
    assert rel_fro(_np(mid["R"]), R) <= 1e-2
    # exactly the product of the BF16-rounded inputs, up to FP32 accumulation
    Ab = sp.csr_matrix((bf16_round(c.A.val), c.A.col, c.A.rowptr), shape=(c.A.rows, c.A.cols))
    Rb = np.asarray(Ab.T @ bf16_round(_np(p16.W)))
    assert elem_rel_max(_np(mid["R"]), Rb) <= 1e-4
    p16.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("K", [100, 200, 400])
def test_c1_full_size_10_sweeps(cuda, K):
    """V = 26,000 x D = 11,000 CSR (the corpus stand-in), 10 sweeps: the
    relative objective after every sweep within 1e-5 of the oracle's, and the
    factors after sweep 10 within 1e-3 (Frobenius), per W column within 2e-3
    and per H row within 1e-3 of the RMS row norm."""
    c = datagen.c1()
    W0, H0 = sparse_init(c, K)
    plan = gpu_plan(c.A, W0, H0, cuda)
    rel = np.array(plan.sweep(10, objective=True))
    print(f"C1 K={K}: GPU sweeps done; running the oracle", flush=True)
    rel_or, facs = oracle_run(c.A, W0, H0, 10)
    d = np.abs(rel - rel_or) / np.array(rel_or)
    print(f"C1 K={K} relative objective difference per sweep:", np.array2string(d, precision=2))
    assert d.max() <= 1e-5, d
    Wg, Hg = _np(plan.W), _np(plan.Ht).T
    Wo, Ho = facs[-1]
    assert rel_fro(Wg, Wo) <= 1e-3 and rel_fro(Hg, Ho) <= 1e-3
    assert col_rel_max(Wg, Wo) <= 2e-3
    assert row_rms_max(Hg, Ho) <= 1e-3
    plan.close()


@pytest.mark.timeout(600)
def test_c1_products_elementwise(cuda):
    """The two sparse products and Grams of one sweep at full size (K = 200),
    element by element against the oracle's products of the same factors."""
    c = datagen.c1()
    K = 200
    W0, H0 = sparse_init(c, K)
    plan = gpu_plan(c.A, W0, H0, cuda)
    Ao = oracle_A(c.A)
    Wn = _np(plan.W)
    plan.half("H")
    mid = plan.intermediates()
    assert elem_rel_max(_np(mid["R"]), np.asarray(Ao.T @ Wn)) <= 1e-4
    assert elem_rel_max(_np(mid["S"]), Wn.T @ Wn) <= 1e-4
    Hn = _np(plan.Ht).T
    plan.half("W")
    mid = plan.intermediates()
    P = np.asarray(Ao @ Hn.T)
    assert elem_rel_max(_np(mid["P"]), P) <= 1e-4
    assert np.all(_np(mid["P"])[np.diff(c.A.rowptr) == 0] == 0.0)
    assert elem_rel_max(_np(mid["Q"]), Hn @ Hn.T) <= 1e-4
    plan.close()


@pytest.mark.timeout(900)
def test_c2_full_size_5_sweeps(cuda):
    """Dense 10^4 x 10^4 image-shaped matrix, K = 240, from the configuration's
    plain U[0,1) init, 5 sweeps: the FP32 path against the oracle after every
    sweep, and the BF16-product path's error against the oracle stated per
    sweep.  This init clips most rows of H to eps in the first sweep (dead
    components whose revival is decided at rounding level), so the 1e-5 bar
    holds for the first sweep; later sweeps are held to the bound a plain FP32
    transcription of Alg. 1 also meets on this problem."""
    A = datagen.c2()
    W0, H0 = datagen.uniform_init(10000, 10000, 240, seed=1)
    plan = gpu_plan(A, W0, H0, cuda)
    r32 = np.array(plan.sweep(5, objective=True))
    plan.close()
    p16 = gpu_plan(A, W0, H0, cuda, precision="bf16")
    r16 = np.array(p16.sweep(5, objective=True))
    p16.close()
    print("C2: GPU sweeps done; running the oracle", flush=True)
    rel_or, _ = oracle_run(A, W0, H0, 5)
    rel_or = np.array(rel_or)
    e32 = np.abs(r32 - rel_or) / rel_or
    e16 = np.abs(r16 - rel_or) / rel_or
    print("C2 fp32 rel-objective error per sweep:", np.array2string(e32, precision=2))
    print("C2 bf16 rel-objective error per sweep:", np.array2string(e16, precision=2))
    assert e32[0] <= 1e-5
    assert e32.max() <= C2_FP32_LATER_BOUND
    assert e16.max() <= BF16_REL_BOUND
    assert np.all(np.isfinite(r16))


@pytest.mark.timeout(900)
def test_c4_w_half_matches_oracle(cuda):
    """10^5 x 3*10^5 CSR, K = 400 (56 column groups spread over XCDs: the
    device-scope norm exchange, four rows per thread): one W half from the
    initial factors, every column against the oracle's W half (P and Q formed
    by the oracle)."""
    c = datagen.c4()
    K = 400
    W0, H0 = sparse_init(c, K)
    plan = gpu_plan(c.A, W0, H0, cuda)
    assert plan.info()["w_groups"] > 32
    plan.half("W")
    Wg = _np(plan.W)
    plan.close()
    print("C4: GPU W half done; running the oracle", flush=True)
    Wo, _, _ = hals.w_half(oracle_A(c.A), hals.normalize_columns(W0), np.asarray(H0, np.float64), EPS)
    print(f"C4 W half: fro {rel_fro(Wg, Wo):.2e}, worst column {col_rel_max(Wg, Wo):.2e}")
    assert rel_fro(Wg, Wo) <= 5e-4
    assert col_rel_max(Wg, Wo) <= 1e-3


@pytest.mark.timeout(600)
def test_c1_plain_uniform_init_properties(cuda):
    """The corpus configuration's own init (plain U[0,1) for W and H, not the
    scale-matched H): what Alg. 1 guarantees at any precision holds -- finite,
    H >= eps, W > 0 with unit columns, objective non-increasing -- and the
    difference from the oracle's trajectory is stated."""
    c = datagen.c1()
    K = 100
    W0, H0 = datagen.uniform_init(c.A.rows, c.A.cols, K, seed=1)
    plan = gpu_plan(c.A, W0, H0, cuda)
    rel = np.array(plan.sweep(5, objective=True))
    Wg, Hg = _np(plan.W), _np(plan.Ht)
    assert np.all(np.isfinite(Wg)) and np.all(np.isfinite(Hg))
    assert Hg.min() >= EPS * (1 - 1e-6) and Wg.min() > 0
    np.testing.assert_allclose(np.linalg.norm(Wg, axis=0), 1.0, rtol=1e-5)
    assert np.all(np.diff(rel) <= 1e-6 * rel[1:])
    rel_or, _ = oracle_run(c.A, W0, H0, 5)
    print("C1 plain init: |rel - rel_oracle| / rel_oracle per sweep:",
          np.array2string(np.abs(rel - rel_or) / np.array(rel_or), precision=2))
    plan.close()


@pytest.mark.timeout(900)
def test_c4_sampled_h_half_and_properties(cuda):
    """10^5 x 3*10^5 CSR, K = 400: every row of the H half is independent, so
    sampled documents are checked exactly against the oracle's H loop; the
    W half is checked by the properties Alg. 1 guarantees."""
    c = datagen.c4()
    K = 400
    V, D = c.A.rows, c.A.cols
    W0, H0 = sparse_init(c, K)
    plan = gpu_plan(c.A, W0, H0, cuda)
    plan.half("H")
    Ht1 = plan.Ht
    rng = np.random.default_rng(0)
    docs = np.sort(rng.choice(D, size=64, replace=False))
    Wn = hals.normalize_columns(W0)
    S = Wn.T @ Wn
    At = c.At.to_scipy().astype(np.float64)
    R = np.asarray(At[docs] @ Wn)                    # rows of A^T W for the sample
    Ho = hals.h_update(H0[:, docs], R, S, EPS)       # H loop on the sampled columns
    got = _np(Ht1[docs]).T
    assert rel_fro(got, Ho) <= 1e-4
    plan.half("W")
    Wg = _np(plan.W)
    assert np.all(np.isfinite(Wg)) and Wg.min() > 0
    np.testing.assert_allclose(np.linalg.norm(Wg, axis=0), 1.0, rtol=1e-4)
    assert _np(plan.Ht).min() >= EPS * (1 - 1e-6)
    _, r1 = plan.objective()
    plan.sweep(1)
    _, r2 = plan.objective()
    assert r2 <= r1 * (1 + 1e-6)
    plan.close()


@pytest.mark.parametrize("K", [16, 200])
def test_bf16_dense_rows_in_p_product(cuda, monkeypatch, K):
    """BF16 products with the densest rows of A taken out of the sparse P
    product and multiplied on the matrix cores in BF16 (NMF_DENSE_ROWS=1 forces
    it at this size): P equals the product of the BF16-rounded inputs up to
    FP32 accumulation, element by element; the objective, whose FP32 P takes
    the same rows through the FP32 matrix-core product, equals the oracle's
    objective of the plan's own factors; eight sweeps stay within the BF16 bar."""
    import scipy.sparse as sp
    monkeypatch.setenv("NMF_DENSE_ROWS", "1")
    c = small_bow()
    lens = np.diff(c.A.rowptr)
    assert np.sum((lens > 128) & (16 * lens >= c.A.cols)) >= 3  # several rows qualify
    W0, H0 = sparse_init(c, K)
    Ao = oracle_A(c.A)
    p16 = gpu_plan(c.A, W0, H0, cuda, precision="bf16")
    p16.half("W")
    Ab = sp.csr_matrix((bf16_round(c.A.val), c.A.col, c.A.rowptr), shape=(c.A.rows, c.A.cols))
    Pb = np.asarray(Ab @ bf16_round(H0.astype(np.float32).astype(np.float64)).T)
    assert elem_rel_max(_np(p16.intermediates()["P"]), Pb) <= 1e-4
    _, rel = p16.objective()
    want = hals.objective(Ao, _np(p16.W), _np(p16.Ht).T)[1]
    assert abs(rel - want) / want <= 1e-5
    p16.close()
    p16 = gpu_plan(c.A, W0, H0, cuda, precision="bf16")
    r16 = np.array(p16.sweep(8, objective=True))
    rel_or, _ = oracle_run(c.A, W0, H0, 8)
    assert np.max(np.abs(r16 - rel_or) / np.array(rel_or)) <= BF16_REL_BOUND
    p16.close()
