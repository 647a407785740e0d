"""Pins of the MU oracle (oracle/mu.py) against what the mathematics fixes:
Lee and Seung's monotonicity, the exact-factorisation fixed point, zeros that
stay zero, the rank-1 limit (the leading singular pair, NumPy's SVD), and the
Karush-Kuhn-Tucker conditions at a limit point."""
import numpy as np
import scipy.sparse as sp

from oracle import hals, mu


def _obj(A, W, H):
    A = A.toarray() if hasattr(A, "toarray") else A
    return 0.5 * float(np.sum((A - W @ H) ** 2))


def test_every_half_step_is_non_increasing():
    rng = np.random.default_rng(0)
    for trial in range(30):
        V, D, K = rng.integers(3, 12), rng.integers(3, 12), rng.integers(1, 5)
        A = rng.random((V, D))
        W, H = rng.random((V, K)), rng.random((K, D))
        f = _obj(A, W, H)
        for _ in range(20):
            H = mu.mu_h(A, W, H, 0.0)
            f1 = _obj(A, W, H)
            assert f1 <= f * (1 + 1e-12)
            W = mu.mu_w(A, W, H, 0.0)
            f2 = _obj(A, W, H)
            assert f2 <= f1 * (1 + 1e-12)
            f = f2


def test_exact_factorisation_is_a_fixed_point():
    rng = np.random.default_rng(1)
    W0, H0 = 0.5 + rng.random((9, 3)), 0.5 + rng.random((3, 7))
    A = W0 @ H0
    W, H = mu.mu_sweep(A, W0, H0, 0.0)
    np.testing.assert_allclose(H, H0, rtol=1e-13)
    np.testing.assert_allclose(W, W0, rtol=1e-13)


def test_zero_entries_stay_zero_and_the_rest_positive():
    rng = np.random.default_rng(2)
    A = rng.random((8, 6))
    W, H = rng.random((8, 3)), rng.random((3, 6))
    H[1, 2] = 0.0
    W[4, 0] = 0.0
    for _ in range(5):
        W, H = mu.mu_sweep(A, W, H, 1e-16)
    assert H[1, 2] == 0.0 and W[4, 0] == 0.0
    mask_h = np.ones_like(H, bool)
    mask_h[1, 2] = False
    mask_w = np.ones_like(W, bool)
    mask_w[4, 0] = False
    assert np.all(H[mask_h] > 0) and np.all(W[mask_w] > 0)


def test_rank_one_reaches_the_leading_singular_value():
    """K = 1 on a positive matrix: the best rank-1 approximation is the leading
    singular pair (non-negative by Perron-Frobenius), objective (||A||^2 - s1^2)/2."""
    rng = np.random.default_rng(3)
    A = 0.1 + rng.random((12, 9))
    W, H = rng.random((12, 1)), rng.random((1, 9))
    for _ in range(400):
        W, H = mu.mu_sweep(A, W, H, 0.0)
    s1 = np.linalg.svd(A, compute_uv=False)[0]
    assert abs(_obj(A, W, H) - 0.5 * (np.sum(A * A) - s1 * s1)) <= 1e-9 * np.sum(A * A)


def test_limit_point_satisfies_kkt():
    """After many iterations on a small problem: gradient >= 0 (up to rounding)
    and complementary slackness H * grad_H = 0, W * grad_W = 0."""
    rng = np.random.default_rng(4)
    A = rng.random((10, 8))
    W, H = rng.random((10, 3)), rng.random((3, 8))
    for _ in range(100000):  # MU approaches its limit slowly
        W, H = mu.mu_sweep(A, W, H, 0.0)
    gH = W.T @ (W @ H - A)
    gW = (W @ H - A) @ H.T
    scale = np.sum(A * A)
    assert np.max(np.abs(H * gH)) <= 1e-6 * scale
    assert np.max(np.abs(W * gW)) <= 1e-6 * scale
    assert gH.min() >= -1e-4 * np.abs(gH).max() and gW.min() >= -1e-4 * np.abs(gW).max()


def test_sparse_and_dense_inputs_agree():
    rng = np.random.default_rng(5)
    Ad = (rng.random((20, 15)) < 0.3) * rng.random((20, 15))
    W, H = rng.random((20, 4)), rng.random((4, 15))
    Wd, Hd = mu.mu_sweep(Ad, W, H, 1e-16)
    Ws, Hs = mu.mu_sweep(sp.csr_matrix(Ad), W, H, 1e-16)
    np.testing.assert_allclose(Ws, Wd, rtol=1e-13)
    np.testing.assert_allclose(Hs, Hd, rtol=1e-13)


def test_hals_converges_faster_than_mu_per_sweep():
    """The qualitative claim of Sec. 6.3 on a small planted problem: after the
    same number of sweeps FAST-HALS has the lower objective."""
    rng = np.random.default_rng(6)
    W0, H0 = rng.random((60, 5)), rng.random((5, 50))
    A = W0 @ H0 + 0.01 * rng.random((60, 50))
    Wi, Hi = rng.random((60, 5)), rng.random((5, 50))
    Wh, Hh = hals.normalize_columns(Wi), Hi.copy()
    Wm, Hm = hals.normalize_columns(Wi), Hi.copy()
    for _ in range(30):
        Wh, Hh = hals.sweep(A, Wh, Hh, 1e-16)
        Wm, Hm = mu.mu_sweep(A, Wm, Hm, 1e-16)
    assert _obj(A, Wh, Hh) < _obj(A, Wm, Hm)
