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


def _hand_network():
    """A network whose outputs are worked out by hand (exact in binary):
    layer 1 copies input i to hidden unit i, bias -1 (negative inputs are
    clipped by the ReLU); layer 2 doubles unit o and adds unit o-1 (not
    symmetric, so a transposed weight matrix shows), bias 0.5 except -10 for
    unit 3 (clipped); layer 3 takes 3 x unit o for logit o, minus unit 12 for
    every logit, bias 0.25 o."""
    W1 = np.zeros((mlp.N_IN, mlp.N_HID))
    W1[np.arange(8), np.arange(8)] = 1.0
    b1 = np.full(mlp.N_HID, -1.0)
    W2 = np.zeros((mlp.N_HID, mlp.N_HID))
    W2[np.arange(64), np.arange(64)] = 2.0
    W2[np.arange(7), np.arange(1, 8)] = 1.0
    b2 = np.full(mlp.N_HID, 0.5)
    b2[3] = -10.0
    W3 = np.zeros((mlp.N_HID, mlp.N_OUT))
    W3[np.arange(12), np.arange(12)] = 3.0
    W3[12, :] = -1.0
    b3 = 0.25 * np.arange(mlp.N_OUT)
    return mlp.pack([W1, b1, W2, b2, W3, b3])


# inputs, and the activations and logits worked out by hand for them
HAND_X = [[3.0, 0.5, 1.0, -2.0, 2.5, 1.25, 7.0, 0.0], [0.0] * 8]
HAND_H1 = [[2.0, 0.0, 0.0, 0.0, 1.5, 0.25, 6.0, 0.0], [0.0] * 8]  # units 8.. are 0
HAND_H2 = [[4.5, 2.5, 0.5, 0.0, 3.5, 2.5, 12.75, 6.5], [0.5, 0.5, 0.5, 0.0, 0.5, 0.5, 0.5, 0.5]]  # units 8.. 0.5
HAND_Z = [[13.0, 7.25, 1.5, 0.25, 11.0, 8.25, 39.25, 20.75, 3.0, 3.25, 3.5, 3.75],
          [1.0, 1.25, 1.5, 0.25, 2.0, 2.25, 2.5, 2.75, 3.0, 3.25, 3.5, 3.75]]


def test_forward_matches_hand_worked_network():
    H1, H2, Z = mlp.forward(_hand_network(), np.array(HAND_X))
    assert np.array_equal(H1[:, :8], HAND_H1) and np.all(H1[:, 8:] == 0.0)
    assert np.array_equal(H2[:, :8], HAND_H2) and np.all(H2[:, 8:] == 0.5)
    assert np.array_equal(Z, HAND_Z)


@pytest.mark.parametrize("mistake", ["no_relu_1", "no_relu_2", "w2_transposed", "no_bias_2", "bias_3_dropped"])
def test_forward_planted_mistakes_miss_the_hand_values(mistake):
    """Each plausible slip in a forward pass changes the hand-worked logits."""
    W1, b1, W2, b2, W3, b3 = mlp.unpack(_hand_network())
    X = np.array(HAND_X)
    a1 = X @ W1 + b1
    H1 = a1 if mistake == "no_relu_1" else np.maximum(a1, 0.0)
    a2 = H1 @ (W2.T if mistake == "w2_transposed" else W2) + (0.0 if mistake == "no_bias_2" else b2)
    H2 = a2 if mistake == "no_relu_2" else np.maximum(a2, 0.0)
    Z = H2 @ W3 + (0.0 if mistake == "bias_3_dropped" else b3)
    assert not np.array_equal(Z, HAND_Z)
