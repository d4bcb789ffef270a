"""Pins for oracle/closed_forms.py and oracle/mc.py: each formula is checked against an
independent route (a library routine, a special case, a second derivation, brute force)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import closed_forms as CF
from oracle import mc
import workloads as W


@pytest.mark.parametrize("a,b,rho", [(0.3, -0.4, 0.5), (-1.2, 0.7, -0.6), (1.5, 1.1, 0.9), (0.0, 0.0, 0.0)])
def test_bivariate_normal_against_scipy(a, b, rho):
    ref = stats.multivariate_normal(mean=[0, 0], cov=[[1, rho], [rho, 1]]).cdf([a, b])
    assert abs(CF.bivariate_normal_cdf(a, b, rho) - ref) < 1e-7


def test_bivariate_normal_identities():
    for a, b, rho in [(0.3, -0.4, 0.5), (-1.2, 0.7, -0.6), (2.0, -0.1, 0.3)]:
        # independence and the reflection identity M(a,b,rho) + M(a,-b,-rho) = Phi(a)
        assert abs(CF.bivariate_normal_cdf(a, b, 0.0) - CF.norm_cdf(a) * CF.norm_cdf(b)) < 1e-14
        s = CF.bivariate_normal_cdf(a, b, rho) + CF.bivariate_normal_cdf(a, -b, -rho)
        assert abs(s - CF.norm_cdf(a)) < 1e-13
        assert abs(CF.bivariate_normal_cdf(a, b, rho) - CF.bivariate_normal_cdf(b, a, rho)) < 1e-13


def test_bs_put_call_parity_and_greeks_by_differences():
    S, K, T, r, s = 105.0, 100.0, 0.7, 0.03, 0.25
    assert abs(CF.bs_call(S, K, T, r, s) - CF.bs_put(S, K, T, r, s) - (S - K * math.exp(-r * T))) < 1e-12
    h = 1e-5
    fd_delta = (CF.bs_call(S * (1 + h), K, T, r, s) - CF.bs_call(S * (1 - h), K, T, r, s)) / (2 * h * S)
    fd_vega = (CF.bs_call(S, K, T, r, s + h) - CF.bs_call(S, K, T, r, s - h)) / (2 * h)
    assert abs(fd_delta - CF.bs_call_delta(S, K, T, r, s)) < 1e-8
    assert abs(fd_vega - CF.bs_vega(S, K, T, r, s)) < 1e-6


def test_one_factor_reduces_to_black_scholes():
    for (S, K, T, r, s) in [(100, 100, 1, 0.05, 0.2), (90, 100, 2, 0.01, 0.35)]:
        for rho in (0.0, 0.4):
            c = CF.one_factor_price([S], K, T, r, [s], rho, "call_max")
            p = CF.one_factor_price([S], K, T, r, [s], rho, "put_max")
            assert abs(c / CF.bs_call(S, K, T, r, s) - 1) < 1e-12
            assert abs(p / CF.bs_put(S, K, T, r, s) - 1) < 1e-12


@pytest.mark.parametrize("S1,S2,s1,s2,rho", [(100, 100, 0.2, 0.3, 0.5), (95, 110, 0.35, 0.15, 0.2),
                                              (120, 85, 0.25, 0.25, 0.0)])
def test_stulz_agrees_with_one_factor(S1, S2, s1, s2, rho):
    K, T, r = 100.0, 1.0, 0.05
    cmax = CF.stulz_call_max(S1, S2, K, T, r, s1, s2, rho)
    cmin = CF.stulz_call_min(S1, S2, K, T, r, s1, s2, rho)
    assert abs(cmax / CF.one_factor_price([S1, S2], K, T, r, [s1, s2], rho, "call_max") - 1) < 1e-12
    assert abs(cmin / CF.one_factor_price([S1, S2], K, T, r, [s1, s2], rho, "call_min") - 1) < 1e-11


def test_call_on_min_at_zero_strike_is_min_forward():
    # e^{-rT} E[min(S1,S2)] = S1 - exchange(S1 -> S2 ... ) computed by Margrabe
    S1, S2, s1, s2, rho, T, r = 100.0, 104.0, 0.2, 0.3, 0.4, 1.3, 0.02
    ref = S1 - CF.margrabe_exchange(S1, S2, T, s1, s2, rho)
    assert abs(CF.stulz_call_min(S1, S2, 1e-9, T, r, s1, s2, rho) - ref) < 1e-8


def test_max_put_call_parity_two_assets():
    S1, S2, s1, s2, rho, K, T, r = 100.0, 100.0, 0.2, 0.3, 0.5, 100.0, 1.0, 0.05
    c = CF.one_factor_price([S1, S2], K, T, r, [s1, s2], rho, "call_max")
    p = CF.one_factor_price([S1, S2], K, T, r, [s1, s2], rho, "put_max")
    ref = CF.discounted_expected_max2(S1, S2, T, s1, s2, rho) - K * math.exp(-r * T)
    assert abs((c - p) - ref) < 1e-10


def test_one_factor_quadrature_converged():
    args = ([95, 100, 110], 100, 0.8, 0.03, [0.25, 0.2, 0.3], 1 / 3)
    a = CF.one_factor_price(*args, "call_max", n_hermite=60)
    b = CF.one_factor_price(*args, "call_max", n_hermite=200)
    assert abs(a / b - 1) < 1e-13


def test_mc_against_closed_forms():
    opt, _ = W.config1()
    v, se = mc.mc_price(opt, 2_000_000, seed=11)
    ref = CF.stulz_call_max(100, 100, 100, 1, 0.05, 0.2, 0.3, 0.5)
    assert abs(v - ref) < 4 * se
    o1 = W.option(1, [100.0], 100.0, 1.0, 0.05, [0.2], [[1.0]])
    v, se = mc.mc_price(o1, 2_000_000, seed=12)
    assert abs(v - CF.bs_call(100, 100, 1, 0.05, 0.2)) < 4 * se
