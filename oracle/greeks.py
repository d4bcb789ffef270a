"""Central finite-difference Greeks of the dense Fourier price at a fixed grid.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

delta_j = dV/dS0_j with S0_j bumped by a relative step h (S0_j (1 +- h));
vega_j  = dV/dsigma_j with sigma_j bumped by an absolute step h; the correlation
matrix is held fixed. The grid (L_k, alpha_k per term) is computed once at the
unbumped parameters and reused, so the derivative is that of the fixed-grid
quadrature (the quantity the GPU adjoint differentiates).

Parity: at d = 1 these reduce to the Black-Scholes delta N(d1) and vega
S0 phi(d1) sqrt(T) (Sec. II, Eq. BSexact), checked in tests/test_oracle_ttcross.py.
"""
from __future__ import annotations

import copy

import numpy as np

from . import fourier


def fixed_grid(opt, N, L=None, alpha=None, tol=fourier.DEFAULT_TOL):
    _, grids = fourier.term_grids(opt, N, L, alpha, tol)
    Ls = np.array([g[0] for g in grids])
    As = np.array([g[1] for g in grids])
    return Ls, As


def fd_greeks(opt, N, L=None, alpha=None, h=1e-4, nthreads=0, tol=fourier.DEFAULT_TOL):
    Ls, As = fixed_grid(opt, N, L, alpha, tol)
    d = opt["d"]
    delta = np.zeros(d)
    vega = np.zeros(d)
    for j in range(d):
        up = copy.deepcopy(opt)
        dn = copy.deepcopy(opt)
        up["S0"][j] *= (1.0 + h)
        dn["S0"][j] *= (1.0 - h)
        pu = fourier.dense_price(up, N, Ls, As, nthreads)
        pd = fourier.dense_price(dn, N, Ls, As, nthreads)
        delta[j] = (pu - pd) / (2.0 * h * opt["S0"][j])
        up = copy.deepcopy(opt)
        dn = copy.deepcopy(opt)
        up["sigma"][j] += h
        dn["sigma"][j] -= h
        pu = fourier.dense_price(up, N, Ls, As, nthreads)
        pd = fourier.dense_price(dn, N, Ls, As, nthreads)
        vega[j] = (pu - pd) / (2.0 * h)
    return delta, vega
