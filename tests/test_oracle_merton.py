"""Pins for the oracle's Merton jump-diffusion (the characteristic-function extension named in
Sec. VI): the dense Fourier sum against the jump-count series (Black-Scholes / Stulz per count),
the series against Monte Carlo, and the jump-free limit."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import fourier as F
from oracle import mc as MC


def _opt2(payoff="call_max"):
    return W.option(2, [95.0, 105.0], 100.0, 1.0, 0.03, [0.2, 0.3], [[1.0, 0.4], [0.4, 1.0]], payoff,
                    jumps=(0.8, [-0.1, 0.05], [[0.02, 0.005], [0.005, 0.03]]))


def test_one_asset_against_the_series():
    o = W.option(1, [100.0], 100.0, 1.0, 0.05, [0.2], [[1.0]], "call_max", jumps=(1.0, [-0.1], [[0.04]]))
    ref = CF.merton_series(o["S0"], o["K"], o["T"], o["r"], o["sigma"], o["corr"], 1.0, [-0.1], [[0.04]])
    p = F.dense_price(o, 256)
    assert abs(p / ref - 1) < 1e-9


@pytest.mark.parametrize("payoff", ["call_max", "call_min"])
def test_two_assets_against_the_series(payoff):
    o = _opt2(payoff)
    ref = CF.merton_series(o["S0"], o["K"], o["T"], o["r"], o["sigma"], o["corr"], o["jump_rate"], o["jump_mean"],
                           o["jump_cov"], payoff)
    p = F.dense_price(o, 192)
    assert abs(p / ref - 1) < 1e-8


def test_series_against_monte_carlo():
    o = _opt2()
    ref = CF.merton_series(o["S0"], o["K"], o["T"], o["r"], o["sigma"], o["corr"], o["jump_rate"], o["jump_mean"],
                           o["jump_cov"], "call_max")
    v, se = MC.mc_price(o, 2_000_000, seed=4)
    assert abs(v - ref) < 4 * se
    # and the martingale condition the compensator enforces: e^{-rT} E[S_T^j] = S0_j
    o1 = W.option(1, [100.0], 1e-9, 1.0, 0.03, [0.2], [[1.0]], "call_max", jumps=(0.8, [-0.1], [[0.02]]))
    v1, se1 = MC.mc_price(o1, 1_000_000, seed=5)
    assert abs(v1 - 100.0) < 4 * se1


def test_no_jumps_is_the_diffusion():
    o = W.random_small_options(1, seed=3, d_choices=(2,))[0]
    z = dict(o, jump_rate=0.0, jump_mean=[0.3, 0.3], jump_cov=[[0.1, 0.0], [0.0, 0.1]])
    assert F.dense_price(z, 64) == F.dense_price(o, 64)
    # jumps of zero size change nothing either (the factor is exp(lambda T (1 - 1)) = 1)
    z0 = dict(o, jump_rate=1.5, jump_mean=[0.0, 0.0], jump_cov=[[0.0, 0.0], [0.0, 0.0]])
    assert abs(F.dense_price(z0, 64) / F.dense_price(o, 64) - 1) < 1e-14


def test_three_assets_against_monte_carlo():
    # a strongly anti-correlated pair with jumps: the grid needs N = 128 here
    o = W.merton_options(1, seed=12, d_choices=(3,), payoffs=("call_max",))[0]
    p = F.dense_price(o, 128)
    v, se = MC.mc_price(o, 2_000_000, seed=6)
    assert abs(p - v) < 4 * se + 1e-4 * abs(v)
