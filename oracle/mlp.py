"""Oracle of the MLP cost model -- TEST INFRASTRUCTURE ONLY (only the tests and
the benchmark's CPU leg use it).

A plain float64 numpy implementation of the network, its loss, its analytic
gradient and one Adam step, written from the definitions:

    h1 = relu(W1 x + b1)        W1: H x I
    h2 = relu(W2 h1 + b2)       W2: H x H
    y  = W3 h2 + b3             W3: O x H
    L  = sum_{b,c} M_bc (y_bc - t_bc)^2 / sum_{b,c} M_bc     (masked mean square)

relu'(z) is taken as 1 for z > 0 and 0 otherwise.  Adam (Kingma and Ba, "Adam: a
method for stochastic optimization", ICLR 2015, Algorithm 1):
    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
    theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Parameters travel as one flat vector in the order W1, b1, W2, b2, W3, b3 (row-major
weights), the same packing the GPU library uses for its inputs and outputs.
"""
from __future__ import annotations

import numpy as np


def sizes(I: int, H: int, O: int):
    return [(H, I), (H,), (H, H), (H,), (O, H), (O,)]


def n_params(I: int, H: int, O: int) -> int:
    return sum(int(np.prod(s)) for s in sizes(I, H, O))


def unpack(theta: np.ndarray, I: int, H: int, O: int):
    out, o = [], 0
    for s in sizes(I, H, O):
        c = int(np.prod(s))
        out.append(np.asarray(theta[o:o + c], dtype=np.float64).reshape(s))
        o += c
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta, X, I, H, O):
    """Returns y (B x O) and the activations needed by the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, I, H, O)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (X, z1, h1, z2, h2)


def loss(y, T, M):
    """Masked mean square error and its gradient with respect to y."""
    M = np.asarray(M, dtype=np.float64)
    cnt = M.sum()
    d = (y - T) * M
    L = float((d * (y - T)).sum() / cnt)
    return L, 2.0 * d / cnt


def backward(theta, cache, dy, I, H, O):
    W1, b1, W2, b2, W3, b3 = unpack(theta, I, H, O)
    X, z1, h1, z2, h2 = cache
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def loss_and_grad(theta, X, T, M, I, H, O):
    y, cache = forward(theta, X, I, H, O)
    L, dy = loss(y, T, M)
    return L, backward(theta, cache, dy, I, H, O)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step at step number t (1-based); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def masked_argmax(y, M):
    """Index of the largest y among the entries with M != 0 (lowest index on ties;
    -1 for a row without any allowed entry)."""
    y = np.where(np.asarray(M) != 0, y, -np.inf)
    idx = np.argmax(y, axis=1)
    idx[np.all(np.asarray(M) == 0, axis=1)] = -1
    return idx


def he_uniform_init(I, H, O, seed):
    """Initial parameters: weights uniform in +-sqrt(6/fan_in) from the seeded
    generator, biases zero (He et al., ICCV 2015, uniform variant)."""
    import synth
    parts = []
    for li, (fo, fi) in enumerate([(H, I), (H, H), (O, H)]):
        lim = np.sqrt(6.0 / fi)
        parts.append(synth.uniform_pm1((fo, fi), seed + li) * lim)
        parts.append(np.zeros(fo))
    return pack(parts)
