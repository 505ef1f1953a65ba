"""FP64 reference of the learned warm-start network (test infrastructure only).

A three-layer perceptron  x -> h -> h -> out  with GELU activations (the erf
form, GELU(z) = z Phi(z)), the mean squared error over all outputs of a batch,
and Adam.  The network is specified by BF16 weights and FP32 accumulation;
its reference here is that specification taken literally:

  bf="weights"  (the reference) the weight matrices are rounded to BF16 (through
                FP32, round to nearest, ties to even); inputs, activations,
                gradients and every sum stay in FP64.  Biases stay in full
                precision.
  bf=False      plain FP64 (finite-difference and closed-form pins).
  bf=True       a diagnostic only: additionally rounds every layer input and each
                backward product's output gradient to BF16, the points where one
                possible kernel design stores them.  It is not a reference, since
                those points are a design choice and not part of the specification.

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


def _rounders(bf):
    """(weight rounding, activation / gradient rounding) of a mode."""
    full = (lambda a: np.asarray(a, dtype=np.float64))
    if bf == "weights":
        return bf16, full
    if bf is True:
        return bf16, bf16
    if bf is False:
        return full, full
    raise ValueError(f"unknown BF16 mode {bf!r}")


def forward(params, shapes, X, bf="weights"):
    """Network output and the cached intermediate values."""
    rw, r = _rounders(bf)
    W1, b1, W2, b2, W3, b3 = unpack(params, shapes)
    A0 = r(X)
    Z1 = A0 @ rw(W1).T + b1
    A1 = r(gelu(Z1))
    Z2 = A1 @ rw(W2).T + b2
    A2 = r(gelu(Z2))
    Y = A2 @ rw(W3).T + b3
    return Y, (A0, Z1, A1, Z2, A2)


def loss_grad(params, shapes, X, T, bf="weights"):
    """Mean squared error sum((Y - T)^2) / Y.size and its gradient (flat, like params),
    with respect to the master weights (the BF16 rounding is taken as identity in the
    backward pass, as usual for low-precision weight copies)."""
    rw, r = _rounders(bf)
    W1, b1, W2, b2, W3, b3 = unpack(params, shapes)
    Y, (A0, Z1, A1, Z2, A2) = forward(params, shapes, X, bf)
    D = Y - T
    loss = float((D * D).sum() / D.size)
    dY = 2.0 * D / D.size
    G3 = r(dY)
    dW3 = G3.T @ A2
    db3 = dY.sum(axis=0)
    dZ2 = (G3 @ rw(W3)) * gelu_grad(Z2)
    G2 = r(dZ2)
    dW2 = G2.T @ A1
    db2 = dZ2.sum(axis=0)
    dZ1 = (G2 @ rw(W2)) * gelu_grad(Z1)
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
