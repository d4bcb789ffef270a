"""Adjoint Greeks (delta, vega) of the GPU tensor-train price against closed forms and
central finite differences of the dense-grid oracle at the same fixed grid."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import fourier as F
from oracle import greeks as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pricer():
    import paper_2203_02804_amd as ttfp
    p = ttfp.Pricer(0)
    yield p
    p.close()


def fixed(opt, N, tol):
    Ls, As = G.fixed_grid(opt, N, tol=tol)
    return Ls, As


def test_d1_black_scholes_greeks(pricer):
    S, K, T, r, s = 100.0, 100.0, 1.0, 0.05, 0.2
    o = W.option(1, [S], K, T, r, [s], [[1.0]], "call_max")
    g = W.grid(128, tol=1e-12, max_rank=4)
    Ls, As = fixed(o, 128, 1e-12)
    prices, delta, vega, status = pricer.price_batch([o], dict(g, L=Ls, alpha=As), greeks=True)
    assert abs(delta[0][0] / CF.bs_call_delta(S, K, T, r, s) - 1) < 1e-8
    assert abs(vega[0][0] / CF.bs_vega(S, K, T, r, s) - 1) < 1e-8


@pytest.mark.parametrize("payoff", ["call_max", "put_max", "call_min"])
def test_d2_greeks_against_oracle_fd(pricer, payoff):
    opt, _ = W.config1(payoff)
    opt = dict(opt, S0=[97.0, 104.0], sigma=[0.22, 0.31])
    N, tol = 64, 1e-11
    Ls, As = fixed(opt, N, tol)
    g = dict(W.grid(N, tol=tol, max_rank=48), L=Ls, alpha=As)
    prices, delta, vega, status = pricer.price_batch([opt], g, greeks=True)
    fd_d, fd_v = G.fd_greeks(opt, N, Ls, As, h=1e-4)
    assert np.allclose(delta[0], fd_d, rtol=1e-6, atol=1e-8 * opt["K"]), (delta[0], fd_d)
    assert np.allclose(vega[0], fd_v, rtol=1e-6, atol=1e-6 * opt["K"]), (vega[0], fd_v)


def test_d3_greeks_random_correlation(pricer):
    # a well-conditioned fixed grid (moderate contour shift) so that the tensor train is
    # accurate relative to the size of the summand, not only to the price
    opt = W.random_small_options(1, seed=61, d_choices=(3,), payoffs=("call_max",))[0]
    N, tol = 64, 1e-11
    g = dict(W.grid(N, tol=tol, max_rank=64), L=14.0, alpha=1.25)
    Ls, As = fixed(opt, N, tol)
    Ls, As = G.fixed_grid(opt, N, 14.0, 1.25)
    prices, delta, vega, status = pricer.price_batch([opt], g, greeks=True)
    assert abs(prices[0] / F.dense_price(opt, N, 14.0, 1.25) - 1) < 1e-9
    fd_d, fd_v = G.fd_greeks(opt, N, Ls, As, h=1e-4)
    assert np.allclose(delta[0], fd_d, rtol=1e-5, atol=1e-7 * opt["K"]), (delta[0], fd_d)
    assert np.allclose(vega[0], fd_v, rtol=1e-5, atol=1e-5 * opt["K"]), (vega[0], fd_v)


def test_batch_greeks_mixed_dimensions(pricer):
    opts = W.random_small_options(5, seed=71, d_choices=(1, 2, 3))
    N, tol = 48, 1e-11
    grids = []
    for o in opts:
        Ls, As = G.fixed_grid(o, N, 12.0, 1.25)
        grids.append(dict(W.grid(N, tol=tol, max_rank=48), L=Ls, alpha=As))
    prices, delta, vega, status = pricer.price_batch(opts, grids, greeks=True)
    for o, g, p, dl, vg in zip(opts, grids, prices, delta, vega):
        ref = F.dense_price(o, N, g["L"], g["alpha"])
        assert abs(p / ref - 1) < 1e-7
        fd_d, fd_v = G.fd_greeks(o, N, g["L"], g["alpha"], h=1e-4)
        assert np.allclose(dl, fd_d, rtol=1e-5, atol=1e-7 * o["K"]), (o, dl, fd_d)
        assert np.allclose(vg, fd_v, rtol=1e-5, atol=1e-5 * o["K"]), (o, vg, fd_v)


def test_autograd_function(pricer):
    import torch

    from paper_2203_02804_amd.autograd import TTPrice, frozen_grids
    opts = W.random_small_options(3, seed=81, d_choices=(2,))
    grid = dict(W.grid(64, tol=1e-12, max_rank=64), L=14.0, alpha=1.25)
    grids = frozen_grids(opts, grid)
    S0 = torch.tensor([o["S0"] for o in opts], dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor([o["sigma"] for o in opts], dtype=torch.float64, device="cuda", requires_grad=True)
    prices = TTPrice.apply(S0, sig, pricer, opts, grids)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    (prices * w).sum().backward()
    _, delta, vega, _ = pricer.price_batch(opts, grids, greeks=True)
    assert np.allclose(S0.grad.cpu().numpy(), np.stack(delta) * w.cpu().numpy()[:, None], rtol=1e-12)
    assert np.allclose(sig.grad.cpu().numpy(), np.stack(vega) * w.cpu().numpy()[:, None], rtol=1e-12)
    # central differences of the GPU price itself (fixed grid) agree with the adjoint
    h = 1e-4
    o = opts[0]
    up = dict(o, S0=[o["S0"][0] * (1 + h), o["S0"][1]])
    dn = dict(o, S0=[o["S0"][0] * (1 - h), o["S0"][1]])
    pu = pricer.price_batch([up], grids[0])[0][0]
    pd = pricer.price_batch([dn], grids[0])[0][0]
    assert abs((pu - pd) / (2 * h * o["S0"][0]) / delta[0][0] - 1) < 1e-5
