"""FP64 oracle of the multiplicative update (MU) baseline (test
infrastructure only; shares no code with the GPU path).

Sec. 2.1 names MU (Lee and Seung) as the simplest NMF algorithm and the
slower-converging comparator of the experiments (Sec. 6.3); the paper does
not print its rules.  For the Frobenius objective of Eq. 2 they are the
Lee-Seung rules, taken here as:

    H <- H * (W^T A) / (W^T W H + delta)
    W <- W * (A H^T) / (W (H H^T) + delta)

(elementwise product and quotient), H first and then W with the new H, as in
one FAST-HALS sweep.  delta > 0 only keeps a zero denominator finite (the
library uses the plan's eps, 1e-16).  Entries that are zero stay zero, and
without delta the objective never increases (Lee and Seung's theorem).
W starts column-normalised, as the library's plans start (it does not change
the method: MU is covariant under W -> W c, H -> H / c)."""
from __future__ import annotations

import numpy as np


def _f64(x):
    if hasattr(x, "toarray") or hasattr(x, "tocsr"):
        return x.astype(np.float64)
    return np.array(x, dtype=np.float64, copy=True)


def mu_h(A, W, H, delta):
    """The H rule: H * (W^T A) / ((W^T W) H + delta)."""
    A, W, H = _f64(A), _f64(W), _f64(H)
    num = np.asarray((A.T @ W).T)
    return H * num / ((W.T @ W) @ H + delta)


def mu_w(A, W, H, delta):
    """The W rule: W * (A H^T) / (W (H H^T) + delta)."""
    A, W, H = _f64(A), _f64(W), _f64(H)
    num = np.asarray(A @ H.T)
    return W * num / (W @ (H @ H.T) + delta)


def mu_sweep(A, W, H, delta):
    """One MU iteration: the H rule, then the W rule with the new H."""
    H = mu_h(A, W, H, delta)
    W = mu_w(A, W, H, delta)
    return W, H
