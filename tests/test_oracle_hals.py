"""Pins of the FP64 FAST-HALS oracle against facts the paper and the
mathematics fix (CPU only).  Each test is chosen so that a plausible slip in
the oracle (a dropped term, a wrong sign or index, a transposed operand, a
missing normalisation) fails at least one of them."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import nnls

from oracle import hals

EPS = 1e-16


def _rand_problem(rng, V, D, K, density=None):
    if density is None:
        A = rng.random((V, D))
    else:
        A = sp.random(V, D, density=density, random_state=rng, format="csr")
        A.data[:] = rng.random(A.nnz) + 0.05
    W = hals.normalize_columns(rng.random((V, K)))
    H = rng.random((K, D))
    return A, W, H


def _dense(A):
    return A.toarray() if hasattr(A, "toarray") else np.asarray(A)


def _f(A, W, H):
    E = _dense(A) - W @ H
    return 0.5 * float(np.sum(E * E))


# ---------------------------------------------------------------- P1 ----
@pytest.mark.parametrize("density", [None, 0.3])
def test_nonnegativity_every_sweep(density):
    """H >= eps and W > 0 (finite) after every sweep; W's columns stay unit norm."""
    rng = np.random.default_rng(11)
    A, W, H = _rand_problem(rng, 40, 30, 6, density)
    for _ in range(15):
        W, H = hals.sweep(A, W, H, EPS)
        assert np.all(np.isfinite(W)) and np.all(np.isfinite(H))
        assert H.min() >= EPS
        assert W.min() > 0.0
        np.testing.assert_allclose(np.linalg.norm(W, axis=0), 1.0, rtol=1e-13)


# ---------------------------------------------------------------- P2 ----
@pytest.mark.parametrize("seed", range(12))
def test_objective_nonincreasing_every_row_and_column_step(seed):
    """With unit-norm columns of W, each H row step is an exact 1-D minimiser and
    each W column step yields the best unit-norm non-negative column, so the
    objective never increases after any single step."""
    rng = np.random.default_rng(100 + seed)
    V, D, K = rng.integers(5, 14), rng.integers(5, 14), rng.integers(1, 5)
    A, W, H = _rand_problem(rng, V, D, K, None if seed % 2 else 0.5)
    f_prev = [_f(A, W, H)]
    worst = [0.0]

    for _ in range(4):
        Wc = W.copy()

        def on_h(k, Hc):
            f = _f(A, Wc, Hc)
            worst[0] = max(worst[0], (f - f_prev[0]) / max(f_prev[0], 1e-300))
            f_prev[0] = f

        H, _, _ = hals.h_half(A, W, H, EPS, on_step=on_h)
        Hc = H.copy()

        def on_w(k, Wn):
            f = _f(A, Wn, Hc)
            worst[0] = max(worst[0], (f - f_prev[0]) / max(f_prev[0], 1e-300))
            f_prev[0] = f

        W, _, _ = hals.w_half(A, W, H, EPS, on_step=on_w)
    assert worst[0] <= 1e-12


def test_objective_can_rise_without_initial_normalisation():
    """Documents why W is column-normalised before the first sweep: without it
    the H step of Alg. 1 (no division by S_kk) is not a minimiser and the
    objective rises on this seeded problem."""
    rng = np.random.default_rng(7)
    A = rng.random((12, 10))
    W = 3.0 * rng.random((12, 3))  # columns far from unit norm
    H = rng.random((3, 10))
    f0 = _f(A, W, H)
    H1, _, _ = hals.h_half(A, W, H, EPS)
    assert _f(A, W, H1) > f0


# ---------------------------------------------------------------- P3 ----
def _golden_min(fun, lo, hi, iters=200):
    """Golden-section search of a unimodal function on [lo, hi]."""
    g = (np.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = fun(c), fun(d)
    for _ in range(iters):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = fun(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = fun(d)
    x = 0.5 * (a + b)
    cands = [lo, x]
    return min(cands, key=fun)


def _brute_min(fun, lo, hi):
    """Dense grid to bracket the minimum, then golden section."""
    grid = np.linspace(lo, hi, 2001)
    vals = np.array([fun(x) for x in grid])
    i = int(np.argmin(vals))
    a, b = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    return _golden_min(fun, a, b)


def test_each_h_entry_is_bruteforce_clipped_minimiser():
    rng = np.random.default_rng(3)
    V, D, K = 5, 4, 3
    A = rng.random((V, D))
    W = hals.normalize_columns(rng.random((V, K)))
    H = rng.random((K, D))
    states = []
    hals.h_half(A, W, H, EPS, on_step=lambda k, Hc: states.append(Hc.copy()))
    Hbefore = H.copy()
    for k in range(K):
        Hnew = states[k]
        for j in range(D):
            # explicit residual with every other row of H at its current value
            rest = A[:, j] - sum(W[:, l] * Hbefore[l, j] for l in range(K) if l != k)

            def fun(h):
                r = rest - W[:, k] * h
                return float(r @ r)

            h_star = _brute_min(fun, EPS, 10.0)
            assert abs(Hnew[k, j] - h_star) <= 1e-7 * max(1.0, abs(h_star))
        Hbefore = Hnew.copy()


def test_each_w_column_is_normalised_bruteforce_minimiser():
    rng = np.random.default_rng(4)
    V, D, K = 4, 6, 3
    A = rng.random((V, D))
    W = hals.normalize_columns(rng.random((V, K)))
    H = rng.random((K, D))
    Q = H @ H.T
    states = []
    hals.w_half(A, W, H, EPS, on_step=lambda k, Wc: states.append(Wc.copy()))
    Wbefore = W.copy()
    for k in range(K):
        col = np.empty(V)
        for v in range(V):
            rest = A[v, :] - sum(Wbefore[v, l] * H[l, :] for l in range(K) if l != k)

            def fun(w):
                r = rest - w * H[k, :]
                return float(r @ r)

            # Alg. 1 clips Q_kk * w at eps, i.e. w at eps / Q_kk
            col[v] = _brute_min(fun, EPS / Q[k, k], 10.0)
        col /= np.linalg.norm(col)
        np.testing.assert_allclose(states[k][:, k], col, rtol=0, atol=1e-7)
        Wbefore = states[k].copy()


def test_w_column_is_best_unit_norm_nonnegative_column():
    """The normalised W column maximises <w, Ptilde> over unit non-negative w
    (V = 2: brute force over the quarter circle)."""
    rng = np.random.default_rng(5)
    V, D, K = 2, 7, 2
    A = rng.random((V, D))
    W = hals.normalize_columns(rng.random((V, K)))
    H = rng.random((K, D))
    W1, _, _ = hals.w_half(A, W, H, EPS, on_step=None)
    # column 0: residual excludes column 0 with the old column 1
    Pt = (A - np.outer(W[:, 1], H[1, :])) @ H[0, :]
    th = np.linspace(0.0, np.pi / 2, 200001)
    cand = np.stack([np.cos(th), np.sin(th)])
    best = cand[:, np.argmax(Pt @ cand)]
    np.testing.assert_allclose(W1[:, 0], best, atol=2e-5)


# ---------------------------------------------------------------- P4 ----
@pytest.mark.parametrize("K", [1, 5, 7, 12])
def test_tiled_equals_untiled_for_every_tile_width(K):
    """Reordering the additions (Sec. 3.3, Alg. 2, Eq. 4-6) changes only rounding."""
    rng = np.random.default_rng(20 + K)
    A, W, H = _rand_problem(rng, 23, 19, K)
    H1, R, S = hals.h_half(A, W, H, EPS)
    W1, P, Q = hals.w_half(A, W, H1, EPS)
    for T in range(1, K + 1):
        Ht = hals.h_update_tiled(H, R, S, EPS, T)
        np.testing.assert_allclose(Ht, H1, rtol=0, atol=1e-12 * np.abs(H1).max())
        Wt = hals.w_update_tiled(W, P, Q, EPS, T)
        np.testing.assert_allclose(Wt, W1, rtol=0, atol=1e-12)


def test_tiled_is_not_trivially_untiled():
    """Guard for the tiled pin: dropping phase 3 (new-tile contributions) must
    break the equality, so the pin really exercises all three phases."""
    rng = np.random.default_rng(31)
    A, W, H = _rand_problem(rng, 15, 11, 6)
    W1, P, Q = hals.w_half(A, W, H, EPS)
    Wt = hals.w_update_tiled(W, P, Q, EPS, 2)
    Q_blockdiag = Q.copy()
    for a in range(0, 6, 2):
        Q_blockdiag[a:a + 2, a + 2:] = 0.0
    Wbad = hals.w_update_tiled(W, P, Q_blockdiag, EPS, 2)
    assert np.abs(Wt - W1).max() < 1e-12
    assert np.abs(Wbad - W1).max() > 1e-6


# ---------------------------------------------------------------- P5 ----
def test_planted_exact_factorisation_is_a_fixed_point():
    rng = np.random.default_rng(8)
    V, D, K = 17, 13, 4
    W0 = rng.random((V, K)) + 0.1
    H0 = rng.random((K, D)) + 0.1
    A = W0 @ H0
    nrm = np.linalg.norm(W0, axis=0)
    W = W0 / nrm
    H = H0 * nrm[:, None]
    W1, H1 = hals.sweep(A, W, H, EPS)
    np.testing.assert_allclose(W1, W, rtol=0, atol=1e-13)
    np.testing.assert_allclose(H1, H, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- P6 ----
def test_planted_separable_recovery():
    """Empirical, seed-pinned: a noise-free separable planted problem is
    recovered (the factorisation is unique up to permutation and scale)."""
    from datagen import planted_separable

    A, W0, H0 = planted_separable(14, 12, 3, seed=9)
    rng = np.random.default_rng(10)
    W = hals.normalize_columns(rng.random((14, 3)))
    H = rng.random((3, 12))
    for _ in range(3000):
        W, H = hals.sweep(A, W, H, EPS)
    _, rel = hals.objective(A, W, H)
    assert rel < 1e-6
    W0n = W0 / np.linalg.norm(W0, axis=0)
    C = W0n.T @ W  # cosines between planted and recovered columns
    perm = np.argmax(C, axis=0)
    assert sorted(perm.tolist()) == [0, 1, 2]
    assert np.all(C[perm, np.arange(3)] > 1 - 1e-6)


# ---------------------------------------------------------------- P7 ----
def test_rank_one_is_power_iteration():
    """K = 1: the W half is W <- A A^T W / ||.||, so W -> u1, H -> s1 v1^T and
    D_F -> (||A||^2 - s1^2) / 2, compared with numpy's SVD."""
    rng = np.random.default_rng(12)
    A = rng.random((9, 7)) + 0.1
    W = hals.normalize_columns(rng.random((9, 1)))
    H = rng.random((1, 7))
    for _ in range(300):
        W, H = hals.sweep(A, W, H, EPS)
    U, s, Vt = np.linalg.svd(A)
    u1 = U[:, 0] * np.sign(U[0, 0])
    v1 = Vt[0] * np.sign(Vt[0, 0])
    np.testing.assert_allclose(W[:, 0], u1, atol=1e-12)
    np.testing.assert_allclose(H[0], s[0] * v1, atol=1e-11)
    f, _ = hals.objective(A, W, H)
    assert abs(f - 0.5 * (np.sum(A * A) - s[0] ** 2)) < 1e-11


# ---------------------------------------------------------------- P8 ----
def test_identity_w_gives_clipped_a():
    rng = np.random.default_rng(13)
    K, D = 5, 9
    A = rng.random((K, D)) - 0.3  # some entries would be negative; clip must catch them
    H = rng.random((K, D))
    H1, R, S = hals.h_half(A, np.eye(K), H, EPS)
    np.testing.assert_allclose(H1, np.maximum(EPS, A), rtol=1e-14, atol=1e-15)


# ---------------------------------------------------------------- P9 ----
def test_foldin_converges_to_nnls():
    """H-only HALS with W fixed is coordinate descent on independent NNLS
    problems, one per column; it must reach scipy's Lawson-Hanson solution."""
    rng = np.random.default_rng(14)
    V, K, Dn = 30, 5, 6
    W = hals.normalize_columns(rng.random((V, K)))
    Anew = rng.random((V, Dn))
    Anew[:, 0] = W @ np.array([1.0, 0.0, 2.0, 0.0, 0.5])  # exact, with zeros
    H = hals.foldin(Anew, W, rng.random((K, Dn)), EPS, 3000)
    for j in range(Dn):
        x, _ = nnls(W, Anew[:, j])
        np.testing.assert_allclose(H[:, j], np.maximum(x, EPS), atol=1e-9)


# ----------------------------------------------------------- objective ----
def test_objective_matches_definition_and_sparse_identity():
    rng = np.random.default_rng(15)
    A, W, H = _rand_problem(rng, 8, 6, 3, density=0.4)
    Ad = A.toarray()
    tot = 0.0
    for v in range(8):
        for d in range(6):
            x = Ad[v, d] - sum(W[v, k] * H[k, d] for k in range(3))
            tot += x * x
    f_d, rel_d = hals.objective(Ad, W, H)
    f_s, rel_s = hals.objective(A, W, H)
    assert abs(f_d - 0.5 * tot) < 1e-12
    assert abs(rel_d - np.sqrt(tot / np.sum(Ad * Ad))) < 1e-12
    assert abs(f_s - f_d) < 1e-12 and abs(rel_s - rel_d) < 1e-12


def test_dead_column_becomes_uniform():
    """A column whose update is <= eps everywhere is eps * 1 after the clip and
    1/sqrt(V) * 1 after normalisation (the formula, followed literally)."""
    rng = np.random.default_rng(16)
    V, K = 11, 3
    W = hals.normalize_columns(rng.random((V, K)))
    Q = np.eye(K) * 2.0
    P = rng.random((V, K))
    P[:, 1] = -5.0
    W1 = hals.w_update(W, P, Q, EPS)
    np.testing.assert_allclose(W1[:, 1], np.full(V, 1 / np.sqrt(V)), rtol=1e-14)
