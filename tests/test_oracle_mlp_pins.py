"""Pins of the MLP oracle: central finite differences of the loss, a one-sample
one-unit network differentiated by hand, the linear regime where the network is
a plain product of matrices, the closed form of Adam's first step, and the
masked arg-max rules."""
import numpy as np
import pytest

import synth
from oracle import mlp


def rand_problem(I, H, O, B, seed):
    theta = mlp.he_uniform_init(I, H, O, seed)
    theta = theta + 0.05 * synth.uniform_pm1(theta.shape, seed + 10)   # non-zero biases
    X = synth.uniform_pm1((B, I), seed + 20)
    T = synth.uniform_pm1((B, O), seed + 21)
    M = (synth.unit(seed + 22, B * O) < 0.7).astype(np.float64).reshape(B, O)
    M[0, 0] = 1.0
    return theta, X, T, M


@pytest.mark.parametrize("I,H,O,B", [(6, 5, 4, 7), (6, 16, 9, 30), (3, 1, 1, 1)])
def test_gradient_matches_central_differences(I, H, O, B):
    theta, X, T, M = rand_problem(I, H, O, B, 100 + H)
    L, g = mlp.loss_and_grad(theta, X, T, M, I, H, O)
    h = 1e-6
    fd = np.zeros_like(theta)
    for p in range(theta.size):
        tp = theta.copy(); tp[p] += h
        tm = theta.copy(); tm[p] -= h
        fd[p] = (mlp.loss_and_grad(tp, X, T, M, I, H, O)[0] -
                 mlp.loss_and_grad(tm, X, T, M, I, H, O)[0]) / (2 * h)
    scale = np.max(np.abs(fd)) + 1e-12
    assert np.max(np.abs(fd - g)) <= 1e-6 * scale
    # a dropped or mis-signed term anywhere shows up in this comparison
    assert np.max(np.abs(g)) > 0


def test_one_sample_one_unit_by_hand():
    """I = H = O = 1: x = 2, W1 = 0.5, b1 = 0.25, W2 = -1.5, b2 = 2, W3 = 3,
    b3 = -1, t = 1, mask 1.
      z1 = 1.25, h1 = 1.25;  z2 = -1.875 + 2 = 0.125, h2 = 0.125;
      y = 0.375 - 1 = -0.625;  L = (y - t)^2 = 2.640625;  dL/dy = 2(y - t) = -3.25
      gW3 = dy h2 = -0.40625, gb3 = -3.25
      dh2 = dy W3 = -9.75, dz2 = -9.75 (z2 > 0): gW2 = dz2 h1 = -12.1875, gb2 = -9.75
      dh1 = dz2 W2 = 14.625, dz1 = 14.625 (z1 > 0): gW1 = dz1 x = 29.25, gb1 = 14.625"""
    theta = np.array([0.5, 0.25, -1.5, 2.0, 3.0, -1.0])
    L, g = mlp.loss_and_grad(theta, np.array([[2.0]]), np.array([[1.0]]), np.array([[1.0]]), 1, 1, 1)
    assert L == 2.640625
    assert np.array_equal(g, [29.25, 14.625, -12.1875, -9.75, -0.40625, -3.25])
    # switch the second unit off (z2 < 0): everything below it gets zero gradient
    theta2 = theta.copy(); theta2[3] = 1.0          # z2 = -0.875
    L2, g2 = mlp.loss_and_grad(theta2, np.array([[2.0]]), np.array([[1.0]]), np.array([[1.0]]), 1, 1, 1)
    assert L2 == 4.0                                 # y = b3 = -1
    assert np.array_equal(g2, [0.0, 0.0, 0.0, 0.0, 0.0, -4.0])


def test_linear_regime_is_a_matrix_product():
    """With positive inputs, non-negative weights and biases every unit is active,
    so y = W3 (W2 (W1 x + b1) + b2) + b3 exactly as composed matrices."""
    I, H, O, B = 6, 8, 5, 10
    parts = [np.abs(synth.uniform_pm1(s, 30 + i)) for i, s in enumerate(mlp.sizes(I, H, O))]
    theta = mlp.pack(parts)
    X = np.abs(synth.uniform_pm1((B, I), 40)) + 0.1
    y, _ = mlp.forward(theta, X, I, H, O)
    W1, b1, W2, b2, W3, b3 = parts
    ref = (W3 @ (W2 @ (W1 @ X.T + b1[:, None]) + b2[:, None]) + b3[:, None]).T
    assert np.allclose(y, ref, rtol=1e-14, atol=0)


def test_adam_first_step_closed_form():
    """At t = 1 the bias corrections give m_hat = g and v_hat = g^2, so each
    parameter moves by lr * g / (|g| + eps)."""
    theta = synth.uniform_pm1((50,), 1)
    g = synth.uniform_pm1((50,), 2)
    g[3] = 0.0
    new, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    assert np.allclose(theta - new, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert new[3] == theta[3]
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_masked_argmax_rules():
    y = np.array([[1.0, 5.0, 3.0, 5.0], [2.0, 2.0, 0.0, -1.0], [9.0, 1.0, 1.0, 1.0]])
    M = np.array([[1, 1, 1, 1], [0, 1, 1, 1], [0, 0, 0, 0]])
    assert list(mlp.masked_argmax(y, M)) == [1, 1, -1]


def test_training_reduces_the_loss():
    I, H, O, B = 6, 16, 7, 64
    theta, X, T, M = rand_problem(I, H, O, B, 7)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0 = mlp.loss_and_grad(theta, X, T, M, I, H, O)[0]
    for t in range(1, 201):
        L, g = mlp.loss_and_grad(theta, X, T, M, I, H, O)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=1e-2)
    assert L < 0.5 * L0
