"""FP64 reference of the learned warm-start network (test infrastructure only).

A three-layer perceptron  x -> h -> h -> out  with GELU activations (the erf
form, GELU(z) = z Phi(z)), the mean squared error over all outputs of a batch,
and Adam.  The GPU path keeps BF16 copies of the weights, rounds each layer's
input and each backward product's output gradient to BF16, and accumulates in
FP32; with bf=True the functions here round at exactly those points (each value
goes to FP32 first, then to BF16 with round-to-nearest-even), so both agree up to
the order and precision of accumulation.  Biases stay in full precision.

Parameter layout (flat): W1 [h, in], b1 [h], W2 [h, h], b2 [h], W3 [out, h], b3 [out].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


def bf16(x):
    """Round to BF16 (through FP32, round to nearest, ties to even); returns float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def sizes_of(n_in, h, n_out):
    return [(h, n_in), (h,), (h, h), (h,), (n_out, h), (n_out,)]


def unpack(params, shapes):
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(np.asarray(params[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(arrs):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrs])


def forward(params, shapes, X, bf=False):
    """Network output and the cached intermediate values."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(params, shapes)
    A0 = r(X)
    Z1 = A0 @ r(W1).T + b1
    A1 = r(gelu(Z1))
    Z2 = A1 @ r(W2).T + b2
    A2 = r(gelu(Z2))
    Y = A2 @ r(W3).T + b3
    return Y, (A0, Z1, A1, Z2, A2)


def loss_grad(params, shapes, X, T, bf=False):
    """Mean squared error sum((Y - T)^2) / Y.size and its gradient (flat, like params)."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(params, shapes)
    Y, (A0, Z1, A1, Z2, A2) = forward(params, shapes, X, bf)
    D = Y - T
    loss = float((D * D).sum() / D.size)
    dY = 2.0 * D / D.size
    G3 = r(dY)
    dW3 = G3.T @ A2
    db3 = dY.sum(axis=0)
    dZ2 = (G3 @ r(W3)) * gelu_grad(Z2)
    G2 = r(dZ2)
    dW2 = G2.T @ A1
    db2 = dZ2.sum(axis=0)
    dZ1 = (G2 @ r(W2)) * gelu_grad(Z1)
    G1 = r(dZ1)
    dW1 = G1.T @ A0
    db1 = dZ1.sum(axis=0)
    return loss, pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) at step t >= 1; returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
