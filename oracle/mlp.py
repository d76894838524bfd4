"""Coordinate network of the learned initial guess, written out plainly in FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU-baseline leg; never by the product library.

Network: h_0 = x, h_{l+1} = tanh(W_l h_l + b_l) for the hidden layers, and a
linear last layer; parameters are packed per layer as W_l (dout x din,
row-major) then b_l.  Loss: the mean of the squared output errors over all
samples and outputs.  Gradient by the chain rule (backpropagation):
  delta_last = 2 (y_hat - y) / count,
  dL/dW_l = delta_l^T h_l,  dL/db_l = sum of delta_l over samples,
  delta_{l-1} = (delta_l W_l) * (1 - h_l^2).
Adam: Kingma & Ba (2015), Algorithm 1, with bias-corrected moments.

bf16=True rounds the two operands of every layer product (h_l and W_l
forward, delta_l and W_l backward) to BF16 (nearest, ties to even) before an
exact product, which is what the matrix-core form of the network computes up
to FP32 summation; the weight gradients are not rounded.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def dims(in_dim: int, width: int, depth: int, out_dim: int) -> List[Tuple[int, int]]:
    """(din, dout) of each layer."""
    d = [in_dim] + [width] * depth + [out_dim]
    return [(d[i], d[i + 1]) for i in range(depth + 1)]


def num_params(ds) -> int:
    return sum(o * i + o for i, o in ds)


def unpack(p: np.ndarray, ds):
    out, k = [], 0
    for i, o in ds:
        W = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((W, b))
    return out


def _bf16(x):
    m, e = np.frexp(np.asarray(x, np.float64))
    return np.ldexp(np.round(m * 256.0), e - 8)


def forward(p: np.ndarray, ds, X: np.ndarray, bf16: bool = False):
    """Returns (output, activations h_0 .. h_L)."""
    r = _bf16 if bf16 else (lambda a: a)
    hs = [np.asarray(X, np.float64)]
    layers = unpack(p, ds)
    for li, (W, b) in enumerate(layers):
        z = r(hs[-1]) @ r(W).T + b
        hs.append(np.tanh(z) if li + 1 < len(layers) else z)
    return hs[-1], hs


def loss_grad(p: np.ndarray, ds, X: np.ndarray, Y: np.ndarray, bf16: bool = False):
    r = _bf16 if bf16 else (lambda a: a)
    out, hs = forward(p, ds, X, bf16)
    diff = out - Y
    loss = float(np.mean(diff ** 2))
    delta = 2.0 * diff / diff.size
    layers = unpack(p, ds)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        gW = delta.T @ hs[li]
        gb = delta.sum(axis=0)
        grads[li] = (gW, gb)
        if li > 0:
            delta = (r(delta) @ r(W)) * (1.0 - hs[li] ** 2)
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, g


def adam(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One step t (1-based) of Adam; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
