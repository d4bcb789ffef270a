"""Merton jump diffusion (the characteristic-function extension of Sec. VI) on the GPU: integrand
entries, prices and Greeks against the oracle's dense grid sums (and its finite differences) on
the same grid, and a ladder."""
import numpy as np
import pytest

import workloads as W
from oracle import fourier as F
from oracle import greeks as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pricer():
    import paper_2203_02804_amd as ttfp
    p = ttfp.Pricer(0)
    yield p
    p.close()


def _grid(opt, N, tol, R, sweeps=8):
    grids = np.array(F.term_grids(opt, N, tol=tol)[1])
    return grids, dict(W.grid(N, tol=tol, max_rank=R, max_sweeps=sweeps), L=grids[:, 0], alpha=grids[:, 1])


def test_integrand_entries(pricer):
    opt = W.merton_options(1, seed=31, d_choices=(3,))[0]
    N = 40
    grids, g = _grid(opt, N, 1e-10, 16)
    rng = np.random.Generator(np.random.PCG64(3))
    idx = rng.integers(0, N, (500, 3))
    for t, term in enumerate(F.terms(opt)):
        gpu = pricer.eval_integrand(opt, g, t, idx)
        ref = F.integrand_at(term, N, grids[t, 0], grids[t, 1], idx)
        assert np.max(np.abs(gpu - ref) / (np.abs(ref) + 1e-300 + 1e-14 * np.max(np.abs(ref)))) < 1e-12


@pytest.mark.parametrize("case", range(5))
def test_prices_against_the_dense_sum(pricer, case):
    opt = W.merton_options(5, seed=32, d_choices=(1, 2, 3))[case]
    N = {1: 128, 2: 96, 3: 48}[opt["d"]]
    # the jump factor raises the ranks above the diffusion's; case 4 (kappa ~ 2.7e4) needs the tighter
    # tolerance for a 1e-8 price and about 20 sweeps to settle
    grids, g = _grid(opt, N, 1e-11, 64, sweeps=16)
    p, ranks, info, rc = pricer.price(opt, g)
    ref = F.dense_price(opt, N, grids[:, 0], grids[:, 1])
    print(f"merton d={opt['d']} {opt['payoff']} lam={opt['jump_rate']:.2f}: rel {p / ref - 1:+.2e} status {rc} "
          f"ranks max {ranks.max()} kappa {info['kappa']:.1e}", flush=True)
    assert rc == 0
    assert abs(p / ref - 1) <= 1e-8


def test_greeks_against_finite_differences(pricer):
    opt = W.merton_options(1, seed=33, d_choices=(2,), payoffs=("call_max",))[0]
    N = 96
    grids, g = _grid(opt, N, 1e-11, 40)
    prices, delta, vega, status = pricer.price_batch([opt], g, greeks=True)
    fd_d, fd_v = G.fd_greeks(opt, N, grids[:, 0], grids[:, 1], h=1e-5)
    print(f"merton greeks: delta {delta[0]} fd {fd_d}; vega {vega[0]} fd {fd_v}", flush=True)
    assert np.allclose(delta[0], fd_d, rtol=1e-5, atol=1e-7)
    assert np.allclose(vega[0], fd_v, rtol=1e-5, atol=1e-6)


def test_ladder_with_jumps(pricer):
    opt = W.merton_options(1, seed=34, d_choices=(2,), payoffs=("call_max",))[0]
    N = 96
    grids, g = _grid(opt, N, 1e-11, 64)
    S0, K, r = W.ladder_points(opt, 12, seed=5)
    prices, info, rc = pricer.price_ladder(opt, g, S0, K, r)
    assert rc == 0
    worst = max(abs(prices[p] / F.dense_price(dict(opt, S0=S0[p].tolist(), K=float(K[p]), r=float(r[p])), N,
                                              grids[:, 0], grids[:, 1]) - 1) for p in range(len(K)))
    print(f"merton ladder: worst rel {worst:.2e}", flush=True)
    assert worst <= 1e-8
