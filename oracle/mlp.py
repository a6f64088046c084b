"""Oracle of the learned cost model's arithmetic: the two-layer perceptron
h = relu(W1 x + b1), y = w2 . h + b2, its mean-squared-error loss, gradient
and Adam step, in float64 numpy.  TEST INFRASTRUCTURE ONLY.

Parameters are one flat array [W1 (H x D, row-major), b1 (H), w2 (H), b2].
``bf16=True`` rounds weights, inputs and hidden activations to bfloat16
(round to nearest even) before use, as the inference kernels do.
"""

import numpy as np


def unpack(P, D, H):
    P = np.asarray(P, dtype=np.float64)
    W1 = P[:H * D].reshape(H, D)
    b1 = P[H * D:H * D + H]
    w2 = P[H * D + H:H * D + 2 * H]
    b2 = P[H * D + 2 * H]
    return W1, b1, w2, b2


def bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(P, X, D, H, bf16_mode=False):
    W1, b1, w2, b2 = unpack(P, D, H)
    X = np.asarray(X, dtype=np.float64)
    if bf16_mode:
        W1, b1, w2, b2 = bf16(W1), bf16(b1), bf16(w2), float(bf16(np.array([b2]))[0])
        X = bf16(X)
    hpre = X @ W1.T + b1
    h = np.maximum(hpre, 0.0)
    if bf16_mode:
        h = bf16(h)
    return h @ w2 + b2, hpre


def loss_grad(P, X, t, D, H):
    """Mean squared error and its gradient with respect to P."""
    W1, b1, w2, b2 = unpack(P, D, H)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    y, hpre = forward(P, X, D, H)
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    h = np.maximum(hpre, 0.0)
    g_w2 = h.T @ dy
    g_b2 = dy.sum()
    dh = np.outer(dy, w2) * (hpre > 0)
    g_W1 = dh.T @ X
    g_b1 = dh.sum(axis=0)
    return loss, np.concatenate([g_W1.ravel(), g_b1, g_w2, [g_b2]])


def adam(P, G, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * G
    v = beta2 * v + (1 - beta2) * G * G
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v
