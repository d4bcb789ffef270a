"""Plain NumPy reference of the price-surrogate MLP (not part of the paper's method).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Network: n_in -> width (x depth, SiLU) -> 1. Parameters are one flat vector: for each layer
(hidden layers, then the head) W [out x in] row-major, then b [out]. The network is defined with
its weights rounded to bfloat16 (round to nearest even: the model stores them so) and everything
else exact: input, activations and sums in float64 (round_weights=False gives the plain float64
network, which the finite-difference pin uses). The gradient is the exact float64 gradient of
the mean squared error, taken through the weight rounding as if it were the identity (the master
weights that the optimiser updates are the unrounded ones).

The GPU kernels differ from this definition only by rounding: they round the input and every
hidden activation (forward) and every hidden dZ (backward) to bfloat16 and accumulate in float32.
rounding_spread measures what such roundings do to the exact network, element by element (the
network itself is never rounded that way here); the GPU tests take their tolerance from it.

Parity: gradient pinned by central finite differences (float64 network); bfloat16 rounding pinned
by torch's bfloat16 conversion; the spread pinned against a deterministic imitation of the
kernels' rounding (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

U_BF16 = 2.0 ** -8           # unit roundoff of bfloat16 (8 significant bits, nearest)
U_F32 = 2.0 ** -24           # unit roundoff of float32


def bf16(x):
    """Round float values to bfloat16 (nearest, ties to even), returned as float64."""
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


def unpack(params, n_in, width, depth, round_weights=True):
    out = []
    off = 0
    for (o, i) in layer_shapes(n_in, width, depth):
        W = np.asarray(params[off:off + o * i], np.float64).reshape(o, i)
        off += o * i
        b = np.asarray(params[off:off + o], np.float64)
        off += o
        out.append((bf16(W) if round_weights else W, b))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, n_in, width, depth, round_weights=True, keep=False):
    layers = unpack(params, n_in, width, depth, round_weights)
    A = np.asarray(x, np.float64)
    Zs, As = [], [A]
    for l in range(depth):
        W, b = layers[l]
        Z = A @ W.T + b
        A = silu(Z)
        Zs.append(Z)
        As.append(A)
    Wh, bh = layers[depth]
    y = A @ Wh[0] + bh[0]
    if keep:
        return y, Zs, As
    return y


def loss(params, x, t, n_in, width, depth, round_weights=True):
    y = forward(params, x, n_in, width, depth, round_weights)
    return float(np.mean((y - t) ** 2))


def grad(params, x, t, n_in, width, depth, round_weights=True):
    """Gradient of the mean squared error with respect to the flat parameter vector."""
    layers = unpack(params, n_in, width, depth, round_weights)
    y, Zs, As = forward(params, x, n_in, width, depth, round_weights, keep=True)
    B = x.shape[0]
    dy = 2.0 * (y - t) / B
    grads = [None] * (depth + 1)
    Wh, _ = layers[depth]
    grads[depth] = ((As[depth].T @ dy)[None, :], np.array([dy.sum()]))
    dZ = dy[:, None] * Wh[0][None, :] * silu_grad(Zs[depth - 1])
    for l in range(depth - 1, -1, -1):
        grads[l] = (dZ.T @ As[l], dZ.sum(axis=0))
        if l > 0:
            W, _ = layers[l]
            dZ = (dZ @ W) * silu_grad(Zs[l - 1])
    return np.concatenate([np.concatenate([g[0].reshape(-1), g[1]]) for g in grads])


def _run(params, x, t, n_in, width, depth, perturb):
    """Forward and gradient of the float64 network with bfloat16 weights, where perturb(v)
    returns v after the relative error of a bfloat16 store (identity: the exact network)."""
    layers = unpack(params, n_in, width, depth, True)
    A = perturb(np.asarray(x, np.float64))
    Zs, As = [], [A]
    for l in range(depth):
        W, b = layers[l]
        Z = A @ W.T + b
        A = perturb(silu(Z))
        Zs.append(Z)
        As.append(A)
    Wh, bh = layers[depth]
    y = A @ Wh[0] + bh[0]
    B = x.shape[0]
    dy = 2.0 * (y - t) / B
    g = [None] * (depth + 1)
    g[depth] = ((As[depth].T @ dy)[None, :], np.array([dy.sum()]))
    dZ = perturb(dy[:, None] * Wh[0][None, :] * silu_grad(Zs[depth - 1]))
    for l in range(depth - 1, -1, -1):
        g[l] = (dZ.T @ As[l], dZ.sum(axis=0))
        if l > 0:
            W, _ = layers[l]
            dZ = perturb((dZ @ W) * silu_grad(Zs[l - 1]))
    return y, np.concatenate([np.concatenate([q[0].reshape(-1), q[1]]) for q in g])


def rounding_spread(params, x, t, n_in, width, depth, draws=16, seed=0):
    """Element-wise spread of the network's output and gradient under the rounding the GPU
    kernels apply where they store bfloat16 values (the input, every hidden activation, every
    hidden dZ): each draw multiplies every such value by (1 + delta), delta uniform on
    [-2^-8, 2^-8] (the relative error of rounding to 8 significant bits), independently. Returns
    the standard deviations over the draws of y (per sample) and of the gradient (per parameter),
    plus the float32 accumulation scale of the gradient (sum over the batch of |dZ| |A| times
    (batch + 2) 2^-24). A GPU result whose roundings behave like one more draw lies within a few
    standard deviations of the exact network, element by element."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pert = lambda v: v * (1.0 + rng.uniform(-U_BF16, U_BF16, size=np.shape(v)))
    ys, gs = [], []
    for _ in range(draws):
        y, g = _run(params, x, t, n_in, width, depth, pert)
        ys.append(y)
        gs.append(g)
    _, gabs = _run_abs(params, x, t, n_in, width, depth)
    return np.std(ys, axis=0, ddof=1), np.std(gs, axis=0, ddof=1), (x.shape[0] + 2) * U_F32 * gabs


def _run_abs(params, x, t, n_in, width, depth):
    """The gradient's terms in absolute value (for the float32 accumulation scale)."""
    layers = unpack(params, n_in, width, depth, True)
    y, Zs, As = forward(params, x, n_in, width, depth, True, keep=True)
    B = x.shape[0]
    dy = np.abs(2.0 * (y - t) / B)
    g = [None] * (depth + 1)
    g[depth] = ((np.abs(As[depth]).T @ dy)[None, :], np.array([dy.sum()]))
    Wh, _ = layers[depth]
    dZ = np.abs(dy[:, None] * Wh[0][None, :] * silu_grad(Zs[depth - 1]))
    for l in range(depth - 1, -1, -1):
        g[l] = (dZ.T @ np.abs(As[l]), dZ.sum(axis=0))
        if l > 0:
            W, _ = layers[l]
            dZ = (dZ @ np.abs(W)) * np.abs(silu_grad(Zs[l - 1]))
    return None, np.concatenate([np.concatenate([q[0].reshape(-1), q[1]]) for q in g])


def simulate_kernel_rounding(params, x, t, n_in, width, depth):
    """The kernels' arithmetic imitated in NumPy (bfloat16 input, activations and dZ; float32
    sums): used only to test the tolerance that rounding_spread gives."""
    layers = unpack(params, n_in, width, depth, True)
    f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)
    A = bf16(x)
    Zs, As = [], [A]
    for l in range(depth):
        W, b = layers[l]
        Z = f32(f32(A @ W.T) + b)
        A = bf16(f32(silu(Z)))
        Zs.append(Z)
        As.append(A)
    Wh, bh = layers[depth]
    y = f32(f32(A @ Wh[0]) + bh[0])
    B = x.shape[0]
    dy = f32(2.0 * (y - t) / B)
    g = [None] * (depth + 1)
    g[depth] = ((As[depth].T @ dy)[None, :], np.array([dy.sum()]))
    dZ = bf16(dy[:, None] * Wh[0][None, :] * silu_grad(Zs[depth - 1]))
    for l in range(depth - 1, -1, -1):
        g[l] = (f32(dZ.T @ As[l]), f32(dZ.sum(axis=0)))
        if l > 0:
            W, _ = layers[l]
            dZ = bf16(f32(dZ @ W) * silu_grad(Zs[l - 1]))
    return y, np.concatenate([np.concatenate([q[0].reshape(-1), q[1]]) for q in g])


def adam_step(params, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    c1 = 1 - b1 ** step
    c2 = 1 - b2 ** step
    return params - lr * (m1 / c1) / (np.sqrt(m2 / c2) + eps), m1, m2
