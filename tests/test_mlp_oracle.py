"""Pins of the oracle's selector network (forward, gradient, Adam) against
facts that do not come from its own code: central finite differences, closed
forms for zero weights and for Adam's first step, and planted mistakes."""
import numpy as np
import pytest

from oracle import mlp


def batch(seed, n=16):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, mlp.N_IN))
    Q = rng.random(size=(n, mlp.N_OUT))
    Q /= Q.sum(axis=1, keepdims=True)
    return X, Q


def test_param_count():
    assert mlp.N_PARAMS == 5516
    assert mlp.init_params(0).shape == (5516,)


def test_zero_parameters_give_uniform_softmax():
    X, Q = batch(1)
    p = np.zeros(mlp.N_PARAMS)
    _, _, Z = mlp.forward(p, X)
    assert np.all(Z == 0)
    assert abs(mlp.loss(p, X, Q) - np.log(12)) < 1e-15


def test_gradient_matches_central_differences():
    X, Q = batch(2)
    p = mlp.init_params(3) * 0.5
    g = mlp.backward(p, X, Q)
    rng = np.random.default_rng(4)
    idx = rng.choice(mlp.N_PARAMS, size=300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, Q) - mlp.loss(p - e, X, Q)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_gradient_sums_to_zero_over_logits_bias():
    # d loss / d b3 = mean(P - Q) sums to 0 over classes (targets are distributions)
    X, Q = batch(5)
    g = mlp.backward(mlp.init_params(6), X, Q)
    gb3 = g[-12:]
    assert abs(gb3.sum()) < 1e-15


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(7)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_planted_mistakes_fail_the_difference_check(monkeypatch):
    X, Q = batch(8)
    p = mlp.init_params(9) * 0.5
    orig = mlp.backward

    def bad_relu_mask(p_, X_, Q_):
        # mistake: drop the ReLU derivative of the first layer
        W1, b1, W2, b2, W3, b3 = mlp.unpack(p_)
        H1, H2, Z = mlp.forward(p_, X_)
        P = np.exp(mlp.log_softmax(Z))
        dZ = (P - Q_) / X_.shape[0]
        dH2 = (dZ @ W3.T) * (H2 > 0)
        dH1 = dH2 @ W2.T
        return mlp.pack([X_.T @ dH1, dH1.sum(0), H1.T @ dH2, dH2.sum(0), H2.T @ dZ, dZ.sum(0)])

    def bad_transpose(p_, X_, Q_):
        g = orig(p_, X_, Q_).copy()
        W3 = mlp.unpack(g)[4]
        g[-12 - 64 * 12:-12] = W3[::-1].ravel()
        return g

    def bad_mean(p_, X_, Q_):
        # mistake: the sum over samples instead of the mean
        return orig(p_, X_, Q_) * X_.shape[0]

    for fn in (bad_relu_mask, bad_transpose, bad_mean):
        g = fn(p, X, Q)
        worst = 0.0
        for i in range(0, mlp.N_PARAMS, 7):
            e = np.zeros_like(p)
            e[i] = 1e-6
            fd = (mlp.loss(p + e, X, Q) - mlp.loss(p - e, X, Q)) / 2e-6
            worst = max(worst, abs(fd - g[i]))
        assert worst > 1e-4
