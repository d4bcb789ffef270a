"""Pins for oracle/ttcross.py (maxvol and the TT-cross sweep) and oracle/greeks.py."""
import itertools
import math

import numpy as np
import pytest

from oracle import closed_forms as CF
from oracle import fourier as F
from oracle import greeks as G
from oracle import ttcross as TT
import workloads as W


@pytest.mark.parametrize("seed", range(6))
def test_maxvol_against_exhaustive_search(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    m, r = int(rng.integers(5, 11)), int(rng.integers(1, 4))
    A = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    delta = 1e-2
    rows, B = TT.maxvol(A, delta=delta)
    assert len(set(rows.tolist())) == r
    # B = A A[rows]^{-1}: identity on the chosen rows, dominated elsewhere
    assert np.allclose(B, A @ np.linalg.inv(A[rows]), atol=1e-12)
    assert np.allclose(B[rows], np.eye(r), atol=1e-12)
    assert np.max(np.abs(B)) <= 1 + delta + 1e-12
    vmax = max(abs(np.linalg.det(A[list(s)])) for s in itertools.combinations(range(m), r))
    v = abs(np.linalg.det(A[rows]))
    # a dominant submatrix has volume >= vmax / ((1+delta)^r r^{r/2}) (Hadamard's inequality on B)
    assert v >= vmax / ((1 + delta) ** r * r ** (r / 2)) - 1e-12


def _grid_fun(funs):
    def f(idx):
        return np.array([funs(row) for row in idx])
    return f


def test_tt_cross_recovers_rank_one_and_rank_two_tensors():
    d, N = 4, 9
    rng = np.random.Generator(np.random.PCG64(1))
    g = rng.standard_normal((d, N)) + 1j * rng.standard_normal((d, N))
    f1 = _grid_fun(lambda i: np.prod([g[k, i[k]] for k in range(d)]))
    cores, info = TT.tt_cross(f1, d, N, max_rank=4, tol=1e-12, seed=2)
    dense = np.prod(g.sum(axis=1))
    assert abs(TT.tt_contract(cores) / dense - 1) < 1e-12
    f2 = _grid_fun(lambda i: sum(g[k, i[k]] for k in range(d)))
    cores, info = TT.tt_cross(f2, d, N, max_rank=4, tol=1e-12, seed=3)
    dense = sum(g[k].sum() * N ** (d - 1) for k in range(d))
    assert abs(TT.tt_contract(cores) / dense - 1) < 1e-12
    idx = rng.integers(0, N, size=(20, d))
    assert np.allclose(TT.tt_value(cores, idx), f2(idx), rtol=1e-11, atol=1e-11)


def test_tt_cross_full_rank_equals_dense_sum():
    opt, _ = W.config1()
    N = 16
    ts, grids = F.term_grids(opt, N, 12.0, 2.0)
    for term, (L, A) in zip(ts, grids):
        fun = lambda idx, term=term, L=L, A=A: F.integrand_at(term, N, L, A, idx)
        cores, info = TT.tt_cross(fun, 2, N, max_rank=N, tol=1e-14, seed=0, eps_rank=0.0)
        s, _ = F.dense_term(term, N, L, A)
        assert abs(TT.tt_contract(cores) / s - 1) < 1e-12


def test_tt_cross_config1_against_dense():
    opt, g = W.config1()
    ref = F.dense_price(opt, 64, 40.0, 2.0)
    ts, grids = F.term_grids(opt, 64, 40.0, 2.0)
    total = 0j
    for t, (term, (L, A)) in enumerate(zip(ts, grids)):
        fun = lambda idx, term=term, L=L, A=A: F.integrand_at(term, 64, L, A, idx)
        cores, info = TT.tt_cross(fun, 2, 64, max_rank=24, tol=1e-10, seed=t)
        total += F.term_scale(opt, L, 64) * TT.tt_contract(cores)
    assert abs(total.real / ref - 1) < 1e-9


def test_fd_greeks_reduce_to_black_scholes():
    S, K, T, r, s = 100.0, 100.0, 1.0, 0.05, 0.2
    o = W.option(1, [S], K, T, r, [s], [[1.0]], "call_max")
    delta, vega = G.fd_greeks(o, 128)
    assert abs(delta[0] / CF.bs_call_delta(S, K, T, r, s) - 1) < 1e-7
    assert abs(vega[0] / CF.bs_vega(S, K, T, r, s) - 1) < 1e-6


def test_fd_greeks_two_assets_against_closed_form_differences():
    S1, S2, s1, s2, rho, K, T, r = 100.0, 95.0, 0.2, 0.3, 0.5, 100.0, 1.0, 0.05
    o = W.option(2, [S1, S2], K, T, r, [s1, s2], W.equicorrelation(2, rho), "call_max")
    delta, vega = G.fd_greeks(o, 96)
    h = 1e-4
    cf = lambda a, b, x, y: CF.stulz_call_max(a, b, K, T, r, x, y, rho)
    d1 = (cf(S1 * (1 + h), S2, s1, s2) - cf(S1 * (1 - h), S2, s1, s2)) / (2 * h * S1)
    v2 = (cf(S1, S2, s1, s2 + h) - cf(S1, S2, s1, s2 - h)) / (2 * h)
    assert abs(delta[0] / d1 - 1) < 1e-7
    assert abs(vega[1] / v2 - 1) < 1e-6
