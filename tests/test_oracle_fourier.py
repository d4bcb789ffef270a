"""Pins for the dense-grid Fourier oracle (oracle/fourier.py + oracle/dense.c)."""
import cmath
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import closed_forms as CF
from oracle import fourier as F
from oracle import mc
import workloads as W


def _xspace_transform(f, z, lo, hi):
    """int_lo^hi e^{i z w} f(w) dw by adaptive quadrature (real and imaginary parts)."""
    re = integrate.quad(lambda w: (cmath.exp(1j * z * w) * f(w)).real, lo, hi, limit=400, epsabs=1e-13)[0]
    im = integrate.quad(lambda w: (cmath.exp(1j * z * w) * f(w)).imag, lo, hi, limit=400, epsabs=1e-13)[0]
    return complex(re, im)


@pytest.mark.parametrize("u", [-3.1, -0.4, 0.0, 0.9, 2.7])
def test_payoff_factor_transforms_by_brute_force(u):
    # call factor (e^w - 1)^+ on Im z > 1
    z = complex(u, 2.5)
    ref = _xspace_transform(lambda w: math.exp(w) - 1.0, z, 0.0, 60.0)
    assert abs(F.payoff_factor(F.KIND_CALL, z) - ref) < 1e-10
    # put factor (1 - e^w)^+ on Im z < 0: same expression
    z = complex(u, -1.3)
    ref = _xspace_transform(lambda w: 1.0 - math.exp(w), z, -60.0, 0.0)
    assert abs(F.payoff_factor(F.KIND_CALL, z) - ref) < 1e-10
    # indicator w < 0 on Im z < 0
    z = complex(u, -0.8)
    ref = _xspace_transform(lambda w: 1.0, z, -80.0, 0.0)
    assert abs(F.payoff_factor(F.KIND_LT, z) - ref) < 1e-10
    # indicator w > 0 on Im z > 0
    z = complex(u, 0.9)
    ref = _xspace_transform(lambda w: 1.0, z, 0.0, 80.0)
    assert abs(F.payoff_factor(F.KIND_GT, z) - ref) < 1e-10


@pytest.mark.parametrize("z", [(complex(0.4, 0.7), complex(-1.1, 0.6)), (complex(2.0, 1.5), complex(0.3, 0.2))])
def test_min_strip_transform_by_brute_force(z):
    # int int e^{i z.w} (min(e^w1, e^w2) - 1)^+ dw over the positive quadrant (the payoff is
    # zero elsewhere), by splitting at w1 = w2: the inner integral is taken in closed form in
    # the larger coordinate and the outer one by adaptive quadrature
    z1, z2 = z

    def inner(w, za, zb):
        # w = the smaller coordinate (in [0, inf)), the larger one runs over (w, inf)
        tail = -cmath.exp(1j * zb * w) / (1j * zb)
        return cmath.exp(1j * za * w) * (math.exp(w) - 1.0) * tail

    hi = 36.0 / (z1.imag + z2.imag - 1.0)            # the integrand decays like e^{-(sum Im z - 1) w}

    def quad_c(f):
        re = integrate.quad(lambda w: f(w).real, 0.0, hi, limit=800, epsabs=1e-14)[0]
        im = integrate.quad(lambda w: f(w).imag, 0.0, hi, limit=800, epsabs=1e-14)[0]
        return complex(re, im)

    ref = quad_c(lambda w: inner(w, z1, z2)) + quad_c(lambda w: inner(w, z2, z1))
    assert abs(F.min_strip_transform(np.array([z1, z2])) - ref) < 1e-10 * max(1.0, abs(ref))
    # the printed form differs from it by the phase i^(d-2) (here 1 at d = 2: they agree)
    assert abs(F.paper_min_transform(np.array([z1, z2])) / F.min_strip_transform(np.array([z1, z2])) - 1) < 1e-13


def test_min_strip_transform_d3_phase_of_the_printed_form():
    z = np.array([complex(0.3, 0.5), complex(-0.7, 0.4), complex(1.2, 0.6)])
    assert abs(F.paper_min_transform(z) / F.min_strip_transform(z) - 1j) < 1e-13


def test_dense_min_strip_against_closed_forms():
    # d = 1: the single-strip transform is the call transform (Black-Scholes)
    o = W.option(1, [100.0], 100.0, 1.0, 0.05, [0.2], [[1.0]], "call_min_strip")
    assert abs(F.dense_price(o, 256) / CF.bs_call(100, 100, 1, 0.05, 0.2) - 1) < 1e-10
    # d = 2: Stulz call on the minimum, priced in one term in asset coordinates
    opt, _ = W.config1("call_min_strip")
    ref = CF.stulz_call_min(100, 100, 100, 1, 0.05, 0.2, 0.3, 0.5)
    assert abs(F.dense_price(opt, 128) / ref - 1) < 1e-9
    # d = 3: the one-factor form, and the term decomposition of the same payoff
    opt = W.option(3, [95.0, 100.0, 110.0], 100.0, 0.8, 0.03, [0.25, 0.2, 0.3], W.equicorrelation(3, 1 / 3),
                   "call_min_strip")
    ref = CF.one_factor_price(opt["S0"], opt["K"], opt["T"], opt["r"], opt["sigma"], 1 / 3, "call_min")
    assert abs(F.dense_price(opt, 96) / ref - 1) < 1e-8
    # the paper's own damping alpha = 5/d on every coordinate converges to the same price; on
    # this grid its larger shift leaves a larger error (8e-5) than the rule's contour
    assert abs(F.dense_price(opt, 96, alpha=5.0 / 3) / ref - 1) < 1e-3
    assert abs(F.dense_price(opt, 256, alpha=5.0 / 3) / ref - 1) < 1e-6


def test_paper_min_transform_does_not_reduce_to_single_asset():
    # As printed (Sec. III.C) the d-dim min transform at d = 1 is -i times the one-asset call transform.
    for z in (complex(0.3, 1.7), complex(-2.0, 3.0)):
        one_asset = -1.0 / (z * (z - 1j))            # Lewis form with K = 1 (Sec. III.B)
        ratio = F.paper_min_transform(np.array([z])) / one_asset
        assert abs(ratio - (-1j)) < 1e-13
        assert abs(F.payoff_factor(F.KIND_CALL, z) / one_asset - 1) < 1e-13


def test_characteristic_function_against_samples():
    opt = W.random_small_options(1, seed=3, d_choices=(3,))[0]
    for term in F.terms(opt):
        rng = np.random.Generator(np.random.PCG64(9))
        n = 400_000
        Wx = rng.multivariate_normal(term["m"], term["C"], size=n)
        for u in (np.array([0.7, -1.1, 0.4]), np.array([-2.0, 0.5, 1.5])):
            emp = np.mean(np.exp(1j * Wx @ u))
            # exp(i u.m - u^T C u / 2) is what dense.c evaluates at z = -u (zero contour shift)
            idx_free = np.exp(1j * u @ term["m"] - 0.5 * u @ term["C"] @ u)
            assert abs(emp - idx_free) < 6 / math.sqrt(n)


def test_integrand_points_match_dense_sum():
    opt = W.random_small_options(1, seed=4, d_choices=(3,))[0]
    N = 12
    ts, grids = F.term_grids(opt, N, 8.0, 1.5)
    for term, (L, A) in zip(ts, grids):
        s, _ = F.dense_term(term, N, L, A)
        idx = np.array(np.unravel_index(np.arange(N ** 3), (N,) * 3)).T
        vals = F.integrand_at(term, N, L, A, idx)
        assert abs(vals.sum() - s) <= 1e-12 * np.abs(vals).sum()


def test_dense_d1_black_scholes():
    for (S, s, T, r) in [(100.0, 0.2, 1.0, 0.05), (80.0, 0.45, 2.0, 0.01)]:
        o = W.option(1, [S], 100.0, T, r, [s], [[1.0]], "call_max")
        assert abs(F.dense_price(o, 128) / CF.bs_call(S, 100.0, T, r, s) - 1) < 1e-10
        o = W.option(1, [S], 100.0, T, r, [s], [[1.0]], "put_max")
        assert abs(F.dense_price(o, 128) / CF.bs_put(S, 100.0, T, r, s) - 1) < 1e-10


def test_dense_d1_paper_hyperparameters():
    # the single-asset experiment's eta = 0.5, alpha = 3 (Sec. V.A): N = 64 nodes -> L = 16
    o = W.option(1, [100.0], 100.0, 1.0, 0.3, [0.5], [[1.0]], "call_max")
    assert abs(F.dense_price(o, 64, 16.0, 3.0) / CF.bs_call(100.0, 100.0, 1.0, 0.3, 0.5) - 1) < 1e-6


def test_dense_config1_against_stulz():
    opt, _ = W.config1()
    stulz = CF.stulz_call_max(100, 100, 100, 1, 0.05, 0.2, 0.3, 0.5)
    g = W.config1_closed_form_grid()
    det = F.dense_price(opt, g["N"], g["L"], g["alpha"], details=True)
    assert abs(det["price"] / stulz - 1) < 1e-12
    assert abs(det["imag"]) < 1e-12 * abs(det["price"])
    assert abs(F.dense_price(opt, 64) / stulz - 1) < 1e-11      # automatic grid
    # literal grid of configuration 1 is aliasing-limited, several percent off
    lit = F.dense_price(opt, 64, 40.0, 2.0)
    assert 1e-2 < abs(lit / stulz - 1) < 1e-1


def test_dense_two_asset_min_and_put():
    opt, _ = W.config1("call_min")
    ref = CF.stulz_call_min(100, 100, 100, 1, 0.05, 0.2, 0.3, 0.5)
    assert abs(F.dense_price(opt, 96) / ref - 1) < 1e-10
    opt, _ = W.config1("put_max")
    cmax = CF.stulz_call_max(100, 100, 100, 1, 0.05, 0.2, 0.3, 0.5)
    ref = cmax - (CF.discounted_expected_max2(100, 100, 1, 0.2, 0.3, 0.5) - 100 * math.exp(-0.05))
    assert abs(F.dense_price(opt, 96) / ref - 1) < 1e-10


@pytest.mark.parametrize("payoff", ["call_max", "put_max", "call_min"])
def test_dense_three_assets_one_factor(payoff):
    opt = W.option(3, [95.0, 100.0, 110.0], 100.0, 0.8, 0.03, [0.25, 0.2, 0.3], W.equicorrelation(3, 1 / 3), payoff)
    ref = CF.one_factor_price(opt["S0"], opt["K"], opt["T"], opt["r"], opt["sigma"], 1 / 3, payoff)
    assert abs(F.dense_price(opt, 96) / ref - 1) < 1e-9


def test_dense_properties():
    opt = W.random_small_options(1, seed=21, d_choices=(3,), payoffs=("call_max",))[0]
    N = 64
    base = F.dense_price(opt, N, details=True)
    assert abs(base["imag"]) < 1e-9 * abs(base["price"])
    # homogeneity: scaling every spot and the strike scales the price
    lam = 1.7
    o2 = dict(opt, S0=[lam * s for s in opt["S0"]], K=lam * opt["K"])
    assert abs(F.dense_price(o2, N) / (lam * base["price"]) - 1) < 1e-10
    # asset permutation invariance
    perm = [2, 0, 1]
    o3 = dict(opt, S0=[opt["S0"][p] for p in perm], sigma=[opt["sigma"][p] for p in perm],
              corr=[[opt["corr"][p][q] for q in perm] for p in perm])
    assert abs(F.dense_price(o3, N) / base["price"] - 1) < 1e-10
    # bounds: max_j BS_j <= C_max <= sum_j BS_j
    bs = [CF.bs_call(opt["S0"][j], opt["K"], opt["T"], opt["r"], opt["sigma"][j]) for j in range(3)]
    assert max(bs) <= base["price"] <= sum(bs)


def test_dense_two_asset_sum_rule():
    # C_max + C_min = BS_1 + BS_2 for any correlation
    for opt in W.random_small_options(3, seed=5, d_choices=(2,), payoffs=("call_max",)):
        cmax = F.dense_price(opt, 96)
        cmin = F.dense_price(dict(opt, payoff="call_min"), 96)
        bs = sum(CF.bs_call(opt["S0"][j], opt["K"], opt["T"], opt["r"], opt["sigma"][j]) for j in range(2))
        assert abs((cmax + cmin) / bs - 1) < 1e-10


@pytest.mark.slow
def test_dense_three_assets_random_correlation_against_mc():
    # brute-force Monte Carlo with 10^8 paths (exact terminal sampling) at d = 3 with a random correlation
    opt = W.random_small_options(1, seed=8, d_choices=(3,), payoffs=("call_max",))[0]
    v, se = mc.mc_price(opt, 100_000_000, seed=3)
    p = F.dense_price(opt, 96)
    assert abs(p - v) < 4 * se
