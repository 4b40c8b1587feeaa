"""Oracle: the parameter-predictor MLP, forward and backward in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

16 standardised matrix features -> 64 (ReLU) -> 64 (ReLU) -> 11 logits split
into three heads (restart: 4 classes, polynomial degree: 5, inner precision:
2); the loss of a sample is the sum of the three softmax cross-entropies, and
the batch loss is their mean.  Parameters are one flat vector in the order
W1 (64 x 16, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (11 x 64), b3 (11).
"""
from __future__ import annotations

import numpy as np

IN, H1, H2 = 16, 64, 64
HEADS = (4, 5, 2)
OUT = sum(HEADS)
SHAPES = [(H1, IN), (H1,), (H2, H1), (H2,), (OUT, H2), (OUT,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)


def unpack(theta: np.ndarray):
    out = []
    o = 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights and zero biases (the seeded draws are an input)."""
    from workloads import he_uniform_params
    return he_uniform_params(seed, SHAPES)


def forward(theta, X, mu, sigma):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Z0 = (X - mu) / sigma
    A1 = Z0 @ W1.T + b1
    H1a = np.maximum(A1, 0.0)
    A2 = H1a @ W2.T + b2
    H2a = np.maximum(A2, 0.0)
    L = H2a @ W3.T + b3
    return L, (Z0, A1, H1a, A2, H2a)


def loss_and_grad(theta, X, mu, sigma, labels):
    """Mean over the batch of the summed head cross-entropies, and its gradient."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    L, (Z0, A1, H1a, A2, H2a) = forward(theta, X, mu, sigma)
    B = X.shape[0]
    dL = np.zeros_like(L)
    loss = 0.0
    o = 0
    for h, k in enumerate(HEADS):
        z = L[:, o:o + k]
        zmax = z.max(axis=1, keepdims=True)
        e = np.exp(z - zmax)
        p = e / e.sum(axis=1, keepdims=True)
        y = labels[:, h]
        loss += float(np.sum(-np.log(p[np.arange(B), y])))
        g = p.copy()
        g[np.arange(B), y] -= 1.0
        dL[:, o:o + k] = g
        o += k
    loss /= B
    dL /= B
    gW3 = dL.T @ H2a
    gb3 = dL.sum(axis=0)
    dH2 = dL @ W3
    dA2 = dH2 * (A2 > 0)
    gW2 = dA2.T @ H1a
    gb2 = dA2.sum(axis=0)
    dH1 = dA2 @ W2
    dA1 = dH1 * (A1 > 0)
    gW1 = dA1.T @ Z0
    gb1 = dA1.sum(axis=0)
    grad = np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, grad


def predict(theta, X, mu, sigma):
    L, _ = forward(theta, X, mu, sigma)
    out = []
    o = 0
    for k in HEADS:
        out.append(np.argmax(L[:, o:o + k], axis=1))
        o += k
    return np.stack(out, axis=1)


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba), bias-corrected; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
