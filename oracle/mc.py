"""Monte Carlo price with exact terminal sampling (Sec. III.A, Eq. mc).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper simulates discretised trajectories; under GBM the terminal law is known
exactly, so S_T^j = S0_j exp((r - sigma_j^2/2) T + sigma_j sqrt(T) (L Z)_j) with
L L^T the correlation matrix and Z standard normal is sampled directly, and the
discounted payoff is averaged. Returns the estimate and its standard error.

Parity: pinned against Black-Scholes and the two-asset closed forms in
tests/test_oracle_closed_forms.py (within 4 standard errors).
"""
from __future__ import annotations

import math

import numpy as np


def payoff(payoff_kind, ST, K):
    if payoff_kind == "call_max":
        return np.maximum(ST.max(axis=1) - K, 0.0)
    if payoff_kind == "put_max":
        return np.maximum(K - ST.max(axis=1), 0.0)
    if payoff_kind in ("call_min", "call_min_strip"):
        return np.maximum(ST.min(axis=1) - K, 0.0)
    raise ValueError(payoff_kind)


def mc_price(opt, n_paths, seed=0, chunk=1 << 20, antithetic=True):
    d = opt["d"]
    S0 = np.asarray(opt["S0"], float)
    sig = np.asarray(opt["sigma"], float)
    Lc = np.linalg.cholesky(np.asarray(opt["corr"], float))
    T, r, K = opt["T"], opt["r"], opt["K"]
    drift = (r - 0.5 * sig ** 2) * T
    vol = sig * math.sqrt(T)
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = float(opt.get("jump_rate", 0.0) or 0.0)
    if lam > 0.0:
        # Merton jumps: a Poisson number of N(muJ, CJ) log-jumps, compensated in the drift
        muJ = np.asarray(opt["jump_mean"], float)
        CJ = np.asarray(opt["jump_cov"], float)
        LJ = np.linalg.cholesky(CJ + 1e-300 * np.eye(d)) if np.any(CJ) else np.zeros((d, d))
        drift = drift - lam * T * (np.exp(muJ + 0.5 * np.diag(CJ)) - 1.0)
        return _mc_jumps(opt["payoff"], S0, K, T, r, drift, vol, Lc, lam, muJ, LJ, n_paths, rng, chunk)
    s1 = 0.0
    s2 = 0.0
    n_done = 0
    m = 0
    while n_done < n_paths:
        n = min(chunk, n_paths - n_done)
        if antithetic:
            h = (n + 1) // 2
            Z = rng.standard_normal((h, d))
            W = Z @ Lc.T
            v = 0.5 * (payoff(opt["payoff"], S0 * np.exp(drift + vol * W), K)
                       + payoff(opt["payoff"], S0 * np.exp(drift - vol * W), K))
            cnt = h
        else:
            Z = rng.standard_normal((n, d))
            v = payoff(opt["payoff"], S0 * np.exp(drift + vol * (Z @ Lc.T)), K)
            cnt = n
        s1 += float(v.sum())
        s2 += float((v * v).sum())
        n_done += n
        m += cnt    # independent samples (an antithetic pair counts once)
    mean = s1 / m
    var = max(s2 / m - mean * mean, 0.0)
    disc = math.exp(-r * T)
    return disc * mean, disc * math.sqrt(var / m)


def _mc_jumps(kind, S0, K, T, r, drift, vol, Lc, lam, muJ, LJ, n_paths, rng, chunk):
    """Plain (non-antithetic) sampling of the jump-diffusion terminal law: given the Poisson count
    n, the jump part is n muJ + sqrt(n) LJ Z'."""
    d = len(S0)
    s1 = s2 = 0.0
    done = 0
    while done < n_paths:
        n = min(chunk, n_paths - done)
        W = rng.standard_normal((n, d)) @ Lc.T
        cnt = rng.poisson(lam * T, n).astype(float)
        J = cnt[:, None] * muJ[None, :] + np.sqrt(cnt)[:, None] * (rng.standard_normal((n, d)) @ LJ.T)
        v = payoff(kind, S0 * np.exp(drift + vol * W + J), K)
        s1 += float(v.sum())
        s2 += float((v * v).sum())
        done += n
    mean = s1 / done
    var = max(s2 / done - mean * mean, 0.0)
    disc = math.exp(-r * T)
    return disc * mean, disc * math.sqrt(var / done)
