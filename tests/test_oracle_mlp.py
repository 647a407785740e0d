"""Pins of the FP64 warm-start network oracle (CPU only): gradients against
central finite differences, activations against their definitions."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import mlp


def _params(rng, K, Hd):
    return {"W1": rng.normal(size=(Hd, K)) * 0.5, "b1": rng.normal(size=Hd) * 0.1,
            "W2": rng.normal(size=(K, Hd)) * 0.5, "b2": rng.normal(size=K) * 0.1}


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    K, Hd, N = 5, 7, 6
    p = _params(rng, K, Hd)
    X = rng.normal(size=(N, K))
    Y = rng.random((N, K))
    _, g = mlp.loss_and_grads(p, X, Y)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2"):
        num = np.zeros_like(p[name])
        it = np.nditer(p[name], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            q1 = {k: v.copy() for k, v in p.items()}
            q2 = {k: v.copy() for k, v in p.items()}
            q1[name][idx] += h
            q2[name][idx] -= h
            num[idx] = (mlp.loss(q1, X, Y) - mlp.loss(q2, X, Y)) / (2 * h)
        err = np.abs(num - g[name]).max() / max(np.abs(num).max(), 1e-12)
        assert err < 1e-6, (name, err)


@pytest.mark.parametrize("z", [-3.0, -0.7, 0.0, 0.4, 2.5])
def test_gelu_is_z_times_gaussian_cdf(z):
    phi = quad(lambda t: math.exp(-0.5 * t * t) / math.sqrt(2 * math.pi), -math.inf, z)[0]
    assert abs(mlp.gelu(z) - z * phi) < 1e-12
    h = 1e-6
    assert abs(mlp.gelu_grad(z) - (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)) < 1e-8


def test_softplus_identities():
    assert abs(mlp.softplus(0.0) - math.log(2.0)) < 1e-15
    z = np.linspace(-15, 15, 31)
    np.testing.assert_allclose(mlp.softplus(z) - mlp.softplus(-z), z, atol=1e-12)
    assert mlp.softplus(25.0) == 25.0  # threshold: identity above 20
    h = 1e-6
    for zz in (-4.0, 0.0, 3.0):
        num = (mlp.softplus(zz + h) - mlp.softplus(zz - h)) / (2 * h)
        assert abs(mlp.softplus_grad(zz) - num) < 1e-8


def test_first_adam_step_closed_form():
    """From zero moments the first step is -lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p = _params(rng, 3, 4)
    g = {k: rng.normal(size=v.shape) for k, v in p.items()}
    st = {}
    p0 = {k: v.copy() for k, v in p.items()}
    mlp.adam_step(p, g, st, lr=1e-2)
    for k in p:
        np.testing.assert_allclose(p[k] - p0[k], -1e-2 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12)


def test_warm_start_is_positively_homogeneous():
    rng = np.random.default_rng(2)
    p = _params(rng, 4, 6)
    R = rng.random((5, 4))
    h1 = mlp.warm_start(p, R, 1e-16)
    h3 = mlp.warm_start(p, 3.0 * R, 1e-16)
    np.testing.assert_allclose(h3, 3.0 * h1, rtol=1e-13)
