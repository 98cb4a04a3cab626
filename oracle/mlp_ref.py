"""FP64 NumPy reference of the proposal MLP (forward, loss, gradient, Adam step).

TEST INFRASTRUCTURE ONLY (used by the tests to check the HIP kernels).
Network: x -> SiLU(W1 x + b1) -> SiLU(W2 . + b2) -> SiLU(W3 . + b3) -> w4 . + b4,
loss = mean((yhat - y)^2).  Inputs are the standardised features; the caller
passes weights and inputs already rounded to bfloat16 when comparing with the
BF16 kernels; everything here is float64.
"""
from __future__ import annotations

import numpy as np

SIZES = [(256, 64), (256, 256), (256, 256)]


def unpack(P):
    P = np.asarray(P, np.float64)
    out, o = [], 0
    for (a, b) in SIZES:
        W = P[o:o + a * b].reshape(a, b); o += a * b
        bb = P[o:o + a]; o += a
        out.append((W, bb))
    w4 = P[o:o + 256]; o += 256
    b4 = P[o]; o += 1
    assert o == P.size
    return out, w4, b4


def pack(layers, w4, b4):
    parts = []
    for W, b in layers:
        parts += [W.ravel(), b]
    parts += [w4, np.array([b4])]
    return np.concatenate(parts)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(P, X):
    layers, w4, b4 = unpack(P)
    h = np.asarray(X, np.float64)
    zs, hs = [], [h]
    for W, b in layers:
        z = h @ W.T + b
        h = silu(z)
        zs.append(z)
        hs.append(h)
    return h @ w4 + b4, zs, hs


def loss_and_grad(P, X, y):
    """Mean squared error and its gradient with respect to the packed parameters."""
    layers, w4, b4 = unpack(P)
    yhat, zs, hs = forward(P, X)
    y = np.asarray(y, np.float64)
    n = y.size
    e = yhat - y
    loss = float(np.mean(e * e))
    dy = 2.0 * e / n
    g_w4 = hs[-1].T @ dy
    g_b4 = dy.sum()
    dh = np.outer(dy, w4)
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        dz = dh * silu_grad(zs[i])
        grads.append((dz.T @ hs[i], dz.sum(0)))
        dh = dz @ layers[i][0]
    grads.reverse()
    return loss, pack(grads, g_w4, g_b4)


def adam_step(P, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) in FP64:
    m <- beta1 m + (1 - beta1) g;  v <- beta2 v + (1 - beta2) g^2;
    P <- P - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
    with t = step >= 1.  Returns the new (P, m, v)."""
    P = np.asarray(P, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return P - lr * mhat / (np.sqrt(vhat) + eps), m, v
