"""Plain NumPy reference of the price-surrogate MLP (not part of the paper's method).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Network: n_in -> width (x depth, SiLU) -> 1. Parameters are one flat vector: for each layer
(hidden layers, then the head) W [out x in] row-major, then b [out].

The precision recipe of the GPU kernels is reproduced so that both can be compared at FP32
level: weights and activations are rounded to bfloat16 (round to nearest even) where the
GPU stores them in bfloat16 (the input, each hidden activation, each hidden dZ, every
weight), products are accumulated in float64 here (FP32 on the GPU). With rounding=False
the same code is exact float64 arithmetic, which the tests pin against central finite
differences of the loss.

Parity: gradient pinned by finite differences (rounding off); bfloat16 rounding pinned by
torch's bfloat16 conversion.
"""
from __future__ import annotations

import numpy as np


def bf16(x, rounding=True):
    """Round float values to bfloat16 (nearest, ties to even), returned as float64."""
    if not rounding:
        return np.asarray(x, np.float64)
    f = np.ascontiguousarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layer_shapes(n_in, width, depth):
    shapes = []
    for l in range(depth + 1):
        i = n_in if l == 0 else width
        o = 1 if l == depth else width
        shapes.append((o, i))
    return shapes


def unpack(params, n_in, width, depth):
    out = []
    off = 0
    for (o, i) in layer_shapes(n_in, width, depth):
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((np.asarray(W, np.float64), np.asarray(b, np.float64)))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, n_in, width, depth, rounding=True, keep=False):
    layers = unpack(params, n_in, width, depth)
    A = bf16(x, rounding)
    Zs, As = [], [A]
    for l in range(depth):
        W, b = layers[l]
        Z = A @ bf16(W, rounding).T + b
        A = bf16(silu(Z), rounding)
        Zs.append(Z)
        As.append(A)
    Wh, bh = layers[depth]
    y = A @ bf16(Wh, rounding)[0] + bh[0]
    if keep:
        return y, Zs, As
    return y


def loss(params, x, t, n_in, width, depth, rounding=True):
    y = forward(params, x, n_in, width, depth, rounding)
    return float(np.mean((y - t) ** 2))


def grad(params, x, t, n_in, width, depth, rounding=True):
    """Gradient of the mean squared error with respect to the flat parameter vector."""
    layers = unpack(params, n_in, width, depth)
    y, Zs, As = forward(params, x, n_in, width, depth, rounding, keep=True)
    B = x.shape[0]
    dy = 2.0 * (y - t) / B
    grads = [None] * (depth + 1)
    Wh, _ = layers[depth]
    grads[depth] = ((As[depth].T @ dy)[None, :], np.array([dy.sum()]))
    dZ = bf16(dy[:, None] * bf16(Wh, rounding)[0][None, :] * silu_grad(Zs[depth - 1]), rounding)
    for l in range(depth - 1, -1, -1):
        gW = dZ.T @ As[l]
        gb = dZ.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            W, _ = layers[l]
            dA = dZ @ bf16(W, rounding)
            dZ = bf16(dA * silu_grad(Zs[l - 1]), rounding)
    return np.concatenate([np.concatenate([g[0].reshape(-1), g[1]]) for g in grads])


def adam_step(params, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    c1 = 1 - b1 ** step
    c2 = 1 - b2 ** step
    return params - lr * (m1 / c1) / (np.sqrt(m2 / c2) + eps), m1, m2
