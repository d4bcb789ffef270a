"""Pins for the CPU reference MLP (oracle/mlp.py)."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def test_bf16_rounding_matches_torch():
    rng = np.random.Generator(np.random.PCG64(0))
    x = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)


def _params(n_in, width, depth, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for (o, i) in M.layer_shapes(n_in, width, depth):
        parts.append(rng.uniform(-1, 1, o * i) * np.sqrt(3.0 / i))
        parts.append(rng.uniform(-0.1, 0.1, o))
    return np.concatenate(parts)


def test_gradient_against_finite_differences():
    n_in, width, depth = 5, 8, 3
    p = _params(n_in, width, depth, 1)
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.standard_normal((17, n_in))
    t = rng.standard_normal(17)
    g = M.grad(p, x, t, n_in, width, depth, round_weights=False)
    h = 1e-6
    for idx in rng.choice(p.size, 40, replace=False):
        e = np.zeros_like(p)
        e[idx] = h
        fd = (M.loss(p + e, x, t, n_in, width, depth, round_weights=False)
              - M.loss(p - e, x, t, n_in, width, depth, round_weights=False)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_parameter_count_of_the_surrogate_shape():
    assert sum(o * i + o for (o, i) in M.layer_shapes(22, 256, 4)) == 203521


def test_adam_first_step_moves_by_lr():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -3.0])
    q, m1, m2 = M.adam_step(p, g, np.zeros(2), np.zeros(2), 1, 0.01)
    assert np.allclose(q, p - 0.01 * np.sign(g), atol=1e-9)


def test_rounding_spread_covers_the_kernels_rounding_points():
    # the kernels' rounding (bfloat16 input, activations, dZ; float32 sums), imitated in NumPy,
    # stays within 8 standard deviations of the rounding spread, element by element; the
    # tolerance is small against the values; a planted mistake is far outside it
    n_in, width, depth = 22, 64, 4
    p = _params(n_in, width, depth, 3)
    rng = np.random.Generator(np.random.PCG64(4))
    x = rng.standard_normal((300, n_in))
    t = np.sin(x[:, :5].sum(axis=1))
    y, gsim = M.simulate_kernel_rounding(p, x, t, n_in, width, depth)
    y0 = M.forward(p, x, n_in, width, depth)
    g0 = M.grad(p, x, t, n_in, width, depth)
    sy, sg, acc = M.rounding_spread(p, x, t, n_in, width, depth, draws=16, seed=5)
    ty, tg = 8 * sy + 1e-6 * np.abs(y0).max(), 8 * sg + acc
    assert np.all(np.abs(y - y0) <= ty)
    assert np.all(np.abs(gsim - g0) <= tg)
    assert np.median(ty) < 1e-2 * np.abs(y0).max()
    assert np.median(tg) < 1e-2 * np.abs(g0).max()
    q = p.copy()
    q[:n_in], q[n_in:2 * n_in] = p[n_in:2 * n_in].copy(), p[:n_in].copy()
    assert np.mean(np.abs(M.forward(q, x, n_in, width, depth) - y0) > ty) > 0.5
    gq = M.grad(q, x, t, n_in, width, depth)
    assert np.mean(np.abs(gq - g0) > tg) > 0.3
