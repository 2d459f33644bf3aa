"""Pins for the fp64 network oracle (no GPU): central finite differences,
closed forms, and a known property of Adam's first step."""
import numpy as np
import pytest

import graphgen

from oracle import mlp


def rand_samples(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, 8))
    T = rng.normal(size=(n, 2))
    return np.hstack([X, T])


@pytest.mark.parametrize("seed", range(4))
def test_gradient_finite_differences(seed):
    w = graphgen.mlp_init_weights(seed)
    S = rand_samples(37, seed + 10)
    loss, g = mlp.loss_and_grad(w, S)
    h = 1e-6
    rng = np.random.default_rng(seed)
    for i in rng.choice(mlp.NPARAMS, 60, replace=False):
        e = np.zeros_like(w)
        e[i] = h
        num = (mlp.loss_and_grad(w + e, S)[0] - mlp.loss_and_grad(w - e, S)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)) + 1e-9, i


def test_closed_form_zero_output_layer():
    w = graphgen.mlp_init_weights(3)
    p = mlp.unpack(w)
    p["W3"][:] = 0.0
    w = mlp.pack(p)
    S = rand_samples(16, 4)
    y, _ = mlp.forward(w, S[:, :8])
    assert np.allclose(y, p["b3"])
    loss, g = mlp.loss_and_grad(w, S)
    T = S[:, 8:]
    assert np.isclose(loss, 0.5 * np.mean(np.sum((p["b3"] - T) ** 2, axis=1)))
    gp = mlp.unpack(g)
    assert np.allclose(gp["b3"], np.mean(p["b3"] - T, axis=0))
    assert np.allclose(gp["W1"], 0) and np.allclose(gp["W2"], 0)


def test_linear_regime_matches_least_squares_gradient():
    """With every pre-activation positive the network is linear in x; the
    output-bias gradient is then the mean residual."""
    w = np.full(mlp.NPARAMS, 0.05)
    X = np.random.default_rng(1).uniform(0.1, 1.0, size=(8, 8))
    S = np.hstack([X, np.zeros((8, 2))])
    y, (_, a1, _, a2, _) = mlp.forward(w, X)
    assert (a1 > 0).all() and (a2 > 0).all()
    _, g = mlp.loss_and_grad(w, S)
    assert np.allclose(mlp.unpack(g)["b3"], y.mean(axis=0))


def test_adam_first_step_moves_by_lr_sign():
    w0 = graphgen.mlp_init_weights(5)
    S = rand_samples(64, 6)
    order = np.arange(64)[None, :]
    w1, _ = mlp.train(S, w0, order, batch=64, lr=1e-3)
    _, g = mlp.loss_and_grad(w0, S)
    big = np.abs(g) > 1e-4
    assert np.allclose((w1 - w0)[big], -1e-3 * np.sign(g[big]), rtol=1e-3)


def test_training_reduces_loss_on_learnable_target():
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 1, size=(512, 8))
    T = np.stack([X[:, 0] * 2 + X[:, 1], 1 - X[:, 2]], axis=1)
    S = np.hstack([X, T])
    order = graphgen.epoch_orders(512, 30, 9)
    w, curve = mlp.train(S, graphgen.mlp_init_weights(1), order, batch=64, lr=3e-3)
    assert curve[-1] < 0.2 * curve[0]
