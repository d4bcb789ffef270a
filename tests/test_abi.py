"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and its
host planning logic (validation, term decomposition, grid rule) agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2203_02804_amd as ttfp
import workloads as W
from oracle import fourier as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ttfp.h")).read()
    return sorted(set(re.findall(r"\b(ttfp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ttfp.load()
    names = declared_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(ttfp.EXPORTS) <= set(names)


def test_strerror():
    lib = ttfp.load()
    assert lib.ttfp_strerror(0) == b"ok"
    assert b"invalid" in lib.ttfp_strerror(-1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_matches_oracle_grid_rule(seed):
    for opt in W.random_small_options(4, seed=seed, d_choices=(1, 2, 3, 5)):
        for N in (64, 128):
            for tol in (1e-8, 1e-12):
                L, A = ttfp.plan(opt, W.grid(N, tol=tol))
                _, grids = F.term_grids(opt, N, tol=tol)
                assert L.shape == (len(grids), opt["d"])
                for t, (Lt, At) in enumerate(grids):
                    assert np.allclose(L[t], Lt, rtol=1e-12)
                    assert np.allclose(A[t], At, rtol=1e-12)


def test_plan_with_jumps_matches_oracle_grid_rule():
    # Merton jumps enter the damping exponent of the rule (the jump cumulant at the shift)
    for opt in W.merton_options(6, seed=21, d_choices=(1, 2, 3)):
        for N in (64, 128):
            L, A = ttfp.plan(opt, W.grid(N, tol=1e-10))
            _, grids = F.term_grids(opt, N, tol=1e-10)
            for t, (Lt, At) in enumerate(grids):
                assert np.allclose(L[t], Lt, rtol=1e-12) and np.allclose(A[t], At, rtol=1e-12)


@pytest.mark.parametrize("bad", [
    dict(jump_rate=-1.0, jump_mean=[0.0, 0.0], jump_cov=[[0.01, 0.0], [0.0, 0.01]]),
    dict(jump_rate=1.0, jump_mean=[0.0, 0.0], jump_cov=[[0.01, 0.02], [0.0, 0.01]]),    # not symmetric
    dict(jump_rate=1.0, jump_mean=[0.0, 0.0], jump_cov=[[0.01, 0.05], [0.05, 0.01]]),   # not semidefinite
    dict(jump_rate=1.0, jump_mean=[float("nan"), 0.0], jump_cov=[[0.01, 0.0], [0.0, 0.01]]),
])
def test_plan_rejects_invalid_jumps(bad):
    opt, g = W.config1()
    with pytest.raises(ttfp.TTFPError):
        ttfp.plan(dict(opt, **bad), g)


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_plan_single_strip_min_matches_oracle(d):
    rng = np.random.Generator(np.random.PCG64(40 + d))
    opt = W.option(d, rng.uniform(85, 115, d), 100.0, 0.9, 0.02, rng.uniform(0.15, 0.35, d),
                   W.sigma_beta(d, 0.5) if d > 1 else [[1.0]], "call_min_strip")
    for N in (50, 128):
        L, A = ttfp.plan(opt, W.grid(N, tol=1e-8))
        _, grids = F.term_grids(opt, N, tol=1e-8)
        assert L.shape == (1, d) and len(grids) == 1
        assert np.allclose(L[0], grids[0][0], rtol=1e-12) and np.allclose(A[0], grids[0][1], rtol=1e-12)
        assert np.all(A > 0) and A.sum() > 1
        # the paper's contour: +5/d on every coordinate
        L, A = ttfp.plan(opt, W.grid(N, tol=1e-8, alpha=5.0 / d))
        assert np.allclose(A, 5.0 / d)
    if d > 1:
        with pytest.raises(ttfp.TTFPError):      # sum of the shifts not above 1
            ttfp.plan(opt, W.grid(64, alpha=0.9 / d))


def test_plan_scalar_grid_signs():
    opt, g = W.config1()
    L, A = ttfp.plan(opt, g)
    assert np.all(L == 40.0)
    assert np.allclose(A, [[2.0, -2.0], [2.0, -2.0]])
    L, A = ttfp.plan(dict(opt, payoff="call_min"), g)
    assert np.allclose(A, [[2.0, 2.0], [2.0, 2.0]])
    L, A = ttfp.plan(dict(opt, payoff="put_max"), g)
    assert np.allclose(A, [[-2.0, -2.0], [-2.0, -2.0]])


@pytest.mark.parametrize("bad", [
    dict(sigma=[0.2, -0.3]),
    dict(S0=[100.0, 0.0]),
    dict(K=-1.0),
    dict(T=0.0),
    dict(corr=[[1.0, 1.2], [1.2, 1.0]]),      # not positive definite
    dict(corr=[[1.0, 0.5], [0.4, 1.0]]),      # not symmetric
    dict(corr=[[0.9, 0.5], [0.5, 1.0]]),      # diagonal not one
    dict(d=0, S0=[], sigma=[], corr=[]),
])
def test_plan_rejects_invalid_options(bad):
    opt, g = W.config1()
    opt = dict(opt, **bad)
    with pytest.raises((ttfp.TTFPError, ValueError)):
        ttfp.plan(opt, g)


def test_plan_rejects_contour_outside_strip():
    opt, g = W.config1()
    with pytest.raises(ttfp.TTFPError):
        ttfp.plan(opt, dict(g, alpha=0.5))        # call coordinate needs alpha > 1
    with pytest.raises(ttfp.TTFPError):
        ttfp.plan(opt, dict(g, N=1))
