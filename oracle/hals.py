"""FP64 FAST-HALS oracle (test infrastructure only; see the package docstring).

Notation follows the paper: A is V x D and non-negative, W is V x K, H is K x D
(this module keeps H in that orientation; the GPU path stores its transpose).

Every function works in float64 on copies of its inputs.  ``A`` may be a dense
ndarray or a ``scipy.sparse`` matrix; library products (``@``) serve as the
matrix-product steps.

Readings of the paper taken here (the GPU path takes the same ones):

* The H row update of Alg. 1 has no division by S_kk; it is the exact 1-D
  minimiser only when every column of W has unit L2 norm.  So the factor W is
  column-normalised once before the first sweep (``normalize_columns``); H is
  left as drawn.
* Normalisation of W happens inside the k loop, column by column, and H is
  never rescaled (Alg. 1, W half).
* Each sweep runs the H half first, then the W half (Alg. 1).
* The clip is max(eps, .) exactly where Alg. 1 places it: on the unit-scale
  value for H, on the Q_kk-scaled value for W.
* When T does not divide K, the tiled update uses ceil(K/T) tiles and a
  narrower last tile.
* Phase 2 adds P (Alg. 2), although Eq. 5 prints it with the subtracted terms.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "normalize_columns",
    "h_update",
    "w_update",
    "h_half",
    "w_half",
    "sweep",
    "objective",
    "h_update_tiled",
    "w_update_tiled",
    "foldin",
    "foldin_objective",
]


def _f64(x):
    if hasattr(x, "toarray") or hasattr(x, "tocsr"):
        return x.astype(np.float64)
    return np.array(x, dtype=np.float64, copy=True)


def normalize_columns(W):
    """Scale every column of W to unit L2 norm (reading of the initialisation
    step of Alg. 1 that makes its H update the exact row minimiser)."""
    W = _f64(W)
    return W / np.sqrt(np.sum(W * W, axis=0, keepdims=True))


def h_update(H, R, S, eps, on_step=None):
    """Alg. 1, H loop: for k = 0..K-1 in order,
    H_k <- max(eps, H_k + R_k - H^T S_k), where H_k is row k of H (1 x D),
    R_k column k of R = A^T W (D x 1) and S_k column k of S = W^T W.
    Rows l < k already hold their new values (Gauss-Seidel order).

    ``on_step(k, H)`` is called after row k is replaced."""
    H = _f64(H)
    R = np.asarray(R, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    K = H.shape[0]
    for k in range(K):
        H[k, :] = np.maximum(eps, H[k, :] + R[:, k] - H.T @ S[:, k])
        if on_step is not None:
            on_step(k, H)
    return H


def w_update(W, P, Q, eps, on_step=None):
    """Alg. 1, W loop: for k = 0..K-1 in order,
    W_k <- max(eps, W_k Q_kk + P_k - W Q_k), then W_k <- W_k / ||W_k||_2,
    where W_k is column k of W, P = A H^T and Q = H H^T.  Columns l < k
    already hold their new, normalised values.

    ``on_step(k, W)`` is called after column k is normalised."""
    W = _f64(W)
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    K = W.shape[1]
    for k in range(K):
        W[:, k] = np.maximum(eps, W[:, k] * Q[k, k] + P[:, k] - W @ Q[:, k])
        W[:, k] = W[:, k] / np.linalg.norm(W[:, k])
        if on_step is not None:
            on_step(k, W)
    return W


def h_half(A, W, H, eps, on_step=None):
    """Alg. 1, H half: R = A^T W, S = W^T W, then ``h_update``.
    Returns (H_new, R, S)."""
    A = _f64(A)
    W = _f64(W)
    R = np.asarray(A.T @ W)
    S = W.T @ W
    return h_update(H, R, S, eps, on_step), R, S


def w_half(A, W, H, eps, on_step=None):
    """Alg. 1, W half: P = A H^T, Q = H H^T (with the new H), then
    ``w_update``.  Returns (W_new, P, Q)."""
    A = _f64(A)
    H = _f64(H)
    P = np.asarray(A @ H.T)
    Q = H @ H.T
    return w_update(W, P, Q, eps, on_step), P, Q


def sweep(A, W, H, eps):
    """One outer iteration of Alg. 1: the H half, then the W half."""
    H, _, _ = h_half(A, W, H, eps)
    W, _, _ = w_half(A, W, H, eps)
    return W, H


def objective(A, W, H):
    """Eq. 2, D_F = 1/2 ||A - W H||_F^2, and the relative objective of
    Sec. 6.2, sqrt(sum (A - WH)^2 / sum A^2).  Returns (D_F, rel).

    Dense A: explicit residual.  Sparse A: the same quantity expanded as
    ||A||^2 - 2 <W, A H^T> + <W^T W, H H^T> in FP64 (W H is never formed)."""
    W = _f64(W)
    H = _f64(H)
    if hasattr(A, "tocsr"):
        A = A.tocsr().astype(np.float64)
        a2 = float(A.multiply(A).sum())
        P = np.asarray(A @ H.T)
        e2 = a2 - 2.0 * float(np.sum(W * P)) + float(np.sum((W.T @ W) * (H @ H.T)))
    else:
        A = np.asarray(A, dtype=np.float64)
        E = A - W @ H
        e2 = float(np.sum(E * E))
        a2 = float(np.sum(A * A))
    e2 = max(e2, 0.0)
    return 0.5 * e2, float(np.sqrt(e2 / a2))


# ------------------------------------------------------- tiled (Alg. 2) ----

def _tiles(K, T):
    """Tile boundaries [start, end) for ceil(K/T) tiles of width T (last one narrower)."""
    return [(s, min(s + T, K)) for s in range(0, K, T)]


def w_update_tiled(W_old, P, Q, eps, T):
    """W half by the three phases of Alg. 2 (Eq. 4-6), tile width T.

    Init: W_new = W_old diag(Q).  Phase 1 (Eq. 4): for each tile tau, the old
    tile tau contributes to all columns left of it.  Then per tile: phase 2
    (in-tile, column by column, old values for columns >= t, new for < t, add
    P, clip at eps, normalise), phase 3 (Eq. 6): the new tile contributes to all
    columns right of it."""
    W_old = _f64(W_old)
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    K = W_old.shape[1]
    tiles = _tiles(K, T)
    W_new = W_old * np.diag(Q)[None, :]
    for (a, b) in tiles:                                  # phase 1
        if a > 0:
            W_new[:, :a] -= W_old[:, a:b] @ Q[a:b, :a]
    for (a, b) in tiles:
        for t in range(a, b):                             # phase 2
            s = W_new[:, a:t] @ Q[t, a:t] + W_old[:, t:b] @ Q[t, t:b]
            W_new[:, t] = np.maximum(eps, W_new[:, t] + P[:, t] - s)
            W_new[:, t] /= np.sqrt(np.sum(W_new[:, t] * W_new[:, t]))
        if b < K:                                         # phase 3
            W_new[:, b:] -= W_new[:, a:b] @ Q[a:b, b:]
    return W_new


def h_update_tiled(H_old, R, S, eps, T):
    """H half by the same three phases without normalisation (the H update is
    done like the W update except for the normalisation, Sec. 4.1).  Works on
    H^T (D x K) so that rows of H play the part of columns of W; the init term
    is H_old itself (coefficient 1, as in Alg. 1's H update)."""
    Ht_old = _f64(H_old).T.copy()
    R = np.asarray(R, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    K = Ht_old.shape[1]
    tiles = _tiles(K, T)
    Y = Ht_old.copy()
    for (a, b) in tiles:                                  # phase 1
        if a > 0:
            Y[:, :a] -= Ht_old[:, a:b] @ S[a:b, :a]
    for (a, b) in tiles:
        for t in range(a, b):                             # phase 2
            s = Y[:, a:t] @ S[t, a:t] + Ht_old[:, t:b] @ S[t, t:b]
            Y[:, t] = np.maximum(eps, Y[:, t] + R[:, t] - s)
        if b < K:                                         # phase 3
            Y[:, b:] -= Y[:, a:b] @ S[a:b, b:]
    return Y.T.copy()


# ------------------------------------------------------------ fold-in ----

def foldin(A_new, W, H0, eps, sweeps, on_sweep=None):
    """H-only FAST-HALS for new columns A_new (V x D') with W fixed: R and S
    are formed once (Alg. 1, H half), then the H loop is repeated ``sweeps``
    times.  ``on_sweep(i, H)`` is called after each repetition."""
    A_new = _f64(A_new)
    W = _f64(W)
    R = np.asarray(A_new.T @ W)
    S = W.T @ W
    H = _f64(H0)
    for i in range(sweeps):
        H = h_update(H, R, S, eps)
        if on_sweep is not None:
            on_sweep(i, H)
    return H


def foldin_objective(A_new, W, H):
    """Relative objective of the fold-in problem, same definition as ``objective``."""
    return objective(A_new, W, H)
