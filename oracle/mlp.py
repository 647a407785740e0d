"""FP64 oracle for the fold-in warm-start network (test infrastructure only).

The paper has no learned component; this network is an extension of the
fold-in step (H-only FAST-HALS with W fixed, the H half of Alg. 1).  Its
definition, fixed here and shared by the GPU path:

    x  = W^T a / ||W^T a||                       (K)
    z1 = W1 x + b1,  g = GELU(z1)                (hidden; GELU(z) = z Phi(z), erf form)
    z2 = W2 g + b2,  y = softplus(z2)            (K; softplus(z) = z for z > 20)
    h0 = ||W^T a|| * y                           (exact rescaling: the NNLS
                                                  solution is positively homogeneous in a)

Loss over a batch of N rows: L = mean over all N*K entries of (y - target)^2.
Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).

Parameters are a dict with W1 [hidden, K], b1 [hidden], W2 [K, hidden], b2 [K].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SOFTPLUS_THRESHOLD = 20.0


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    cdf = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def softplus(z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z > SOFTPLUS_THRESHOLD, z, np.log1p(np.exp(np.minimum(z, SOFTPLUS_THRESHOLD))))


def softplus_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z > SOFTPLUS_THRESHOLD, 1.0, 1.0 / (1.0 + np.exp(-z)))


def forward(params, X):
    """Returns (y, cache) for inputs X [N, K]."""
    X = np.asarray(X, dtype=np.float64)
    W1 = np.asarray(params["W1"], dtype=np.float64)
    b1 = np.asarray(params["b1"], dtype=np.float64)
    W2 = np.asarray(params["W2"], dtype=np.float64)
    b2 = np.asarray(params["b2"], dtype=np.float64)
    z1 = X @ W1.T + b1
    g = gelu(z1)
    z2 = g @ W2.T + b2
    y = softplus(z2)
    return y, (X, z1, g, z2)


def loss(params, X, Y):
    y, _ = forward(params, X)
    d = y - np.asarray(Y, dtype=np.float64)
    return float(np.mean(d * d))


def loss_and_grads(params, X, Y):
    """MSE loss and its gradients with respect to W1, b1, W2, b2."""
    y, (X, z1, g, z2) = forward(params, X)
    Y = np.asarray(Y, dtype=np.float64)
    n_el = y.size
    d = y - Y
    L = float(np.mean(d * d))
    dy = 2.0 * d / n_el
    dz2 = dy * softplus_grad(z2)
    W2 = np.asarray(params["W2"], dtype=np.float64)
    gW2 = dz2.T @ g
    gb2 = dz2.sum(axis=0)
    dg = dz2 @ W2
    dz1 = dg * gelu_grad(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return L, {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2}


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place on FP64 copies; ``state`` holds m, v and step t."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for name in ("W1", "b1", "W2", "b2"):
        g = np.asarray(grads[name], dtype=np.float64)
        m = state.setdefault("m_" + name, np.zeros_like(g))
        v = state.setdefault("v_" + name, np.zeros_like(g))
        m[...] = beta1 * m + (1.0 - beta1) * g
        v[...] = beta2 * v + (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        params[name] = np.asarray(params[name], dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return params


def warm_start(params, R, eps):
    """h0 per row of R = A_new^T W (rows = new documents): the network applied
    to the L2-normalised row, rescaled by the row norm; rows with zero norm get
    eps.  Result clipped below at eps like every H entry."""
    R = np.asarray(R, dtype=np.float64)
    nrm = np.sqrt(np.sum(R * R, axis=1, keepdims=True))
    safe = np.where(nrm > 0, nrm, 1.0)
    y, _ = forward(params, R / safe)
    h0 = np.where(nrm > 0, nrm * y, 0.0)
    return np.maximum(eps, h0)
