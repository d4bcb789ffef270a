"""GPU surrogate kernels (BF16 MFMA forward/backward, Adam) against the CPU reference MLP,
and the surrogate's gate / TT fallback on TT-generated prices."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def net():
    from paper_2203_02804_amd.surrogate import MLP
    n = MLP(22, 256, 4, n_models=2, max_batch=4096, seed=7)
    yield n
    n.close()


def _xt(B, seed):
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((B, 22)).astype(np.float32)
    t = np.sin(x[:, :5].sum(axis=1)).astype(np.float32)
    return x, t, torch.tensor(x, device="cuda").contiguous(), torch.tensor(t, device="cuda").contiguous()


@pytest.mark.parametrize("B", [1, 37, 1000])
def test_forward_matches_reference(net, B):
    x, t, xd, td = _xt(B, B)
    for model in range(2):
        p = net.get_params(model).astype(np.float64)
        gpu = net.forward(model, xd).double().cpu().numpy()
        ref = M.forward(p, x.astype(np.float64), 22, 256, 4)
        scale = np.max(np.abs(ref)) + 1e-30
        # FP32 accumulation order and rare bfloat16 rounding ties differ from the reference
        assert np.median(np.abs(gpu - ref)) <= 1e-5 * scale
        assert np.max(np.abs(gpu - ref)) <= 1e-2 * scale


def test_gradient_matches_reference(net):
    x, t, xd, td = _xt(512, 3)
    p = net.get_params(0).astype(np.float64)
    g, loss = net.grad(0, xd, td)
    ref = M.grad(p, x.astype(np.float64), t.astype(np.float64), 22, 256, 4)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert rel < 1e-2, rel
    assert abs(loss - np.mean((M.forward(p, x.astype(np.float64), 22, 256, 4) - t) ** 2)) < 1e-4 * (1 + loss)


def test_adam_step_matches_reference(net):
    x, t, xd, td = _xt(256, 4)
    p0 = net.get_params(1).astype(np.float64)
    g, _ = net.grad(1, xd, td)
    net.train_step(1, xd, td, 1e-3)
    p1 = net.get_params(1).astype(np.float64)
    ref, _, _ = M.adam_step(p0, g.astype(np.float64), np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    assert np.max(np.abs(p1 - ref)) < 1e-6
    net.set_params(1, p0.astype(np.float32))      # restore (and reset the optimizer state)


def test_training_reduces_loss():
    import torch

    from paper_2203_02804_amd.surrogate import MLP
    n = MLP(22, 256, 4, n_models=1, max_batch=2048, seed=11)
    x, t, xd, td = _xt(2048, 5)
    first = n.train_step(0, xd, td, 1e-3)
    for _ in range(300):
        last = n.train_step(0, xd, td, 1e-3)
    assert last < 0.1 * first
    n.close()


def test_surrogate_gate_and_fallback():
    import paper_2203_02804_amd as ttfp
    from paper_2203_02804_amd.surrogate import Surrogate
    pricer = ttfp.Pricer(0)
    # one-factor correlations, where the TT labels are accurate to ~1e-7 at this grid and rank
    grid = W.grid(128, tol=1e-8, max_rank=48, max_sweeps=4)
    opts = W.config5_options(1536, seed=5, corr_kind="beta")
    prices, status = pricer.price_batch(opts, grid)
    sur = Surrogate(d=5, n_models=4, max_batch=4096, seed=1)
    info = sur.fit(opts[:1280], prices[:1280], steps=1500, batch=512, lr=2e-3, holdout=0.15)
    test = opts[1280:]
    ref = prices[1280:]
    mean, spread = sur.predict(test)
    rel = np.abs(mean / ref - 1)
    assert np.median(rel) < 0.15                      # trained on ~1100 prices: usable, not precise
    # a gate that lets about a third of the rows through: the calibrated error estimate
    # bounds the actual error of the served rows (checked against their TT prices)
    est = sur.factor * spread / np.abs(mean)
    gate = float(np.quantile(est, 0.3))
    out, ok = sur.price(test, pricer, grid, rel_gate=gate)
    assert ok.sum() > 0
    assert np.mean(np.abs(out[ok] / ref[ok] - 1) <= gate) > 0.8
    # rows that failed the gate carry TT prices
    fb = ~ok
    if fb.any():
        assert np.allclose(out[fb], ref[fb], rtol=1e-4)
    # gate 0: everything falls back to TT
    out0, ok0 = sur.price(test, pricer, grid, rel_gate=0.0)
    assert not ok0.any()
    assert np.allclose(out0, ref, rtol=1e-4)
    pricer.close()
