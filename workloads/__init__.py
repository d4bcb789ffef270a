"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws market parameters and grid settings. It contains none of
the pricing arithmetic (no characteristic function, payoff transform, grid rule
or tensor-train step), so the oracle and the GPU path can both take their inputs
from here without sharing any of the method.

An option is a plain dict:

    d        number of assets
    S0       spot prices, list of d floats
    K        strike
    T        maturity in years
    r        continuously compounded risk-free rate
    sigma    volatilities, list of d floats
    corr     correlation matrix, d x d nested list (symmetric, unit diagonal, SPD)
    payoff   "call_max" | "put_max" | "call_min" | "call_min_strip" (the call on the minimum
             priced in the paper's own form: one term in asset coordinates)

A grid setting is a dict with N (nodes per dimension), L and alpha (None means
"let the pricer choose"), tol, max_rank, max_sweeps and seed.

Workloads follow the market model of the paper (correlated geometric Brownian
motion, Sec. II.A) and its correlation family Sigma(beta) (Sec. V.B, Eq. covmat);
the random-correlation configurations use a normalised Wishart draw.
"""
from __future__ import annotations

import numpy as np

PAYOFFS = ("call_max", "put_max", "call_min")
# the call on the minimum in the paper's own form: asset coordinates, one term, the joint
# single-strip transform (not drawn by the random generators, whose streams stay as they were)
ALL_PAYOFFS = PAYOFFS + ("call_min_strip",)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def equicorrelation(d: int, rho: float) -> list:
    """Unit-diagonal matrix with rho off the diagonal."""
    c = np.full((d, d), float(rho))
    np.fill_diagonal(c, 1.0)
    return c.tolist()


def sigma_beta(d: int, beta: float) -> list:
    """The paper's one-parameter family (beta |+><+| + 1)/(1+beta) (Sec. V.B, Eq. covmat):
    ones on the diagonal and beta/(1+beta) off it."""
    return equicorrelation(d, beta / (1.0 + beta))


def wishart_correlation(rng: np.random.Generator, d: int, dof: int, lam_floor: float = 0.05) -> list:
    """A ~ N(0,1)^{d x dof}, W = A A^T, R = D^{-1/2} W D^{-1/2}; redrawn while the
    smallest eigenvalue of R is below lam_floor."""
    while True:
        a = rng.standard_normal((d, dof))
        w = a @ a.T
        s = 1.0 / np.sqrt(np.diag(w))
        r = w * s[:, None] * s[None, :]
        r = 0.5 * (r + r.T)
        np.fill_diagonal(r, 1.0)
        if np.linalg.eigvalsh(r)[0] >= lam_floor:
            return r.tolist()


def option(d, S0, K, T, r, sigma, corr, payoff="call_max", jumps=None) -> dict:
    """jumps: None, or (rate, mean[d], cov[d][d]) of Merton's log-jump sizes (Sec. VI)."""
    if payoff not in ALL_PAYOFFS:
        raise ValueError(payoff)
    o = dict(d=int(d), S0=[float(x) for x in S0], K=float(K), T=float(T), r=float(r),
             sigma=[float(x) for x in sigma], corr=[[float(x) for x in row] for row in corr],
             payoff=payoff)
    if jumps is not None:
        lam, mu, cov = jumps
        o.update(jump_rate=float(lam), jump_mean=[float(x) for x in mu], jump_cov=[[float(x) for x in row] for row in cov])
    return o


def merton_options(n, seed=11, d_choices=(1, 2, 3), payoffs=("call_max", "call_min", "put_max")):
    """Random options with Merton jumps: the market draws of random_small_options, a jump rate
    U[0.2, 2] per year, log-jump means U[-0.2, 0.1] and a log-jump covariance 0.1^2 x (a
    Sigma(beta) matrix, beta U[0, 1]) scaled by U[0.5, 2] per asset."""
    rng = _rng(seed)
    out = []
    for o in random_small_options(n, seed=seed + 1000, d_choices=d_choices, payoffs=payoffs):
        d = o["d"]
        s = 0.1 * rng.uniform(0.5, 2.0, d)
        cov = np.asarray(sigma_beta(d, rng.uniform(0.0, 1.0))) * np.outer(s, s)
        out.append(dict(o, jump_rate=float(rng.uniform(0.2, 2.0)), jump_mean=rng.uniform(-0.2, 0.1, d).tolist(),
                        jump_cov=cov.tolist()))
    return out


def grid(N, L=None, alpha=None, tol=1e-8, max_rank=32, max_sweeps=6, seed=0) -> dict:
    return dict(N=int(N), L=L, alpha=alpha, tol=float(tol), max_rank=int(max_rank),
                max_sweeps=int(max_sweeps), seed=int(seed))


# --- configuration 1: d=2 call on max, literal market and grid -------------------------------

def config1(payoff="call_max"):
    """S0=(100,100), K=100, T=1, r=0.05, vols (0.2,0.3), rho=0.5.
    Literal grid: N=64 per dimension on [-40,40], |alpha|=2, tol 1e-10, max rank 8."""
    opt = option(2, [100.0, 100.0], 100.0, 1.0, 0.05, [0.2, 0.3], equicorrelation(2, 0.5), payoff)
    return opt, grid(64, L=40.0, alpha=2.0, tol=1e-10, max_rank=8)


def config1_closed_form_grid():
    """The grid on which configuration 1 resolves the closed form: N=256, L=40, |alpha|=3."""
    return grid(256, L=40.0, alpha=3.0, tol=1e-10, max_rank=64)


# --- configuration 2: d=5 call on max with random parameters ---------------------------------

def _draw_d5(rng, d, corr_kind, beta=0.5, dof=None):
    sigma = rng.uniform(0.1, 0.4, size=d)
    S0 = rng.uniform(80.0, 120.0, size=d)
    T = rng.uniform(0.25, 2.0)
    if corr_kind == "wishart":
        corr = wishart_correlation(rng, d, dof if dof else 2 * d)
    else:
        corr = sigma_beta(d, beta)
    return option(d, S0, 100.0, T, 0.03, sigma, corr, "call_max")


def config2(seed=2203, corr_kind="wishart"):
    """d=5 call on max: vols ~ U[0.1,0.4], S0 ~ U[80,120], T ~ U[0.25,2], Wishart
    correlation with 10 degrees of freedom (or Sigma(0.5) for corr_kind='beta'),
    K=100, r=0.03; N=128, tol 1e-8, max rank 32."""
    rng = _rng(seed)
    return _draw_d5(rng, 5, corr_kind), grid(128, tol=1e-8, max_rank=32)


def config2_batch(n, seed=2203, corr_kind="wishart", d=5):
    """n independent options drawn from configuration 2's distributions."""
    rng = _rng(seed)
    return [_draw_d5(rng, d, corr_kind) for _ in range(n)]


def config3(seed=2804, corr_kind="wishart"):
    """d=20 call on max from the same distributions; N=256, tol 1e-8, max rank 64."""
    rng = _rng(seed)
    return _draw_d5(rng, 20, corr_kind), grid(256, tol=1e-8, max_rank=64)


# --- configuration 4: the batched book --------------------------------------------------------

def config4(n=8192, seed=22030):
    """Book of n call-on-max options: d ~ U{2..10}, N ~ U{64,128,256}, S0_j = 100,
    K = 100 U[0.8,1.2], T ~ U[0.1,3], vols ~ U[0.1,0.5], Wishart correlation with 2d
    degrees of freedom, r = 0.03. Returns (options, Ns)."""
    rng = _rng(seed)
    opts, Ns = [], []
    for _ in range(n):
        d = int(rng.integers(2, 11))
        N = int(rng.choice([64, 128, 256]))
        K = 100.0 * rng.uniform(0.8, 1.2)
        T = rng.uniform(0.1, 3.0)
        sigma = rng.uniform(0.1, 0.5, size=d)
        corr = wishart_correlation(rng, d, 2 * d)
        opts.append(option(d, [100.0] * d, K, T, 0.03, sigma, corr, "call_max"))
        Ns.append(N)
    return opts, Ns


# --- configuration 5: surrogate training/inference inputs -------------------------------------

def config5_options(n, seed=5, corr_kind="wishart"):
    """d=5 call-on-max options for the price surrogate: vols ~ U[0.1,0.4], S0 ~ U[80,120],
    K = 100, T ~ U[0.25,2], r ~ U[0,0.06], Wishart correlation (10 dof), or for
    corr_kind='beta' the family Sigma(beta) with beta ~ U[0,1]."""
    rng = _rng(seed)
    out = []
    for _ in range(n):
        sigma = rng.uniform(0.1, 0.4, size=5)
        S0 = rng.uniform(80.0, 120.0, size=5)
        T = rng.uniform(0.25, 2.0)
        r = rng.uniform(0.0, 0.06)
        if corr_kind == "wishart":
            corr = wishart_correlation(rng, 5, 10)
        else:
            corr = sigma_beta(5, rng.uniform(0.0, 1.0))
        out.append(option(5, S0, 100.0, T, r, sigma, corr, "call_max"))
    return out


def random_small_options(n, seed, d_choices=(1, 2, 3), payoffs=PAYOFFS):
    """Small random options (d <= 3) for property and parity tests."""
    rng = _rng(seed)
    out = []
    for _ in range(n):
        d = int(rng.choice(d_choices))
        sigma = rng.uniform(0.15, 0.4, size=d)
        S0 = rng.uniform(85.0, 115.0, size=d)
        T = rng.uniform(0.5, 1.5)
        r = rng.uniform(0.0, 0.05)
        corr = wishart_correlation(rng, d, 3 * d) if d > 1 else [[1.0]]
        pay = str(rng.choice(list(payoffs))) if d > 1 else str(rng.choice(["call_max", "put_max"]))
        out.append(option(d, S0, 100.0, T, r, sigma, corr, pay))
    return out


# --- the paper's multi-asset experiment (Sec. V.B, Table I and the bond-dimension study) --------
# grid spacing eta of Table I by dimension (0.2 for the dimensions the table does not list)
PAPER_TABLE_ETA = {2: 0.5, 3: 0.4, 4: 0.3, 5: 0.3, 6: 0.2, 7: 0.2, 8: 0.2, 9: 0.2, 10: 0.2, 15: 0.2}
PAPER_TABLE_DIMS = (2, 3, 4, 5, 6, 7, 8, 9, 10, 15)


def paper_experiment(d, beta=0.5, tol=1e-10, max_rank=64, max_sweeps=8, seed=0, N=50, eta=None):
    """The call on the minimum of d assets of the paper's experiment: r = 0.3, sigma = 0.5, T = 1,
    S0 = K = 100 on every asset, correlation Sigma(beta), priced in asset coordinates with the
    single-strip transform on N nodes (the paper's 50) of spacing eta (Table I's by default;
    L = N eta / 2) and the shift alpha = 5 / d on every coordinate. Returns (option, grid)."""
    opt = option(d, [100.0] * d, 100.0, 1.0, 0.3, [0.5] * d, sigma_beta(d, beta), "call_min_strip")
    eta = PAPER_TABLE_ETA.get(d, 0.2) if eta is None else eta
    return opt, grid(N, L=N * eta / 2, alpha=5.0 / d, tol=tol, max_rank=max_rank, max_sweeps=max_sweeps, seed=seed)


# --- market ladders: one option's volatilities, correlation and maturity at many (S0, K, r) -----
def ladder_points(opt, n, seed=7, spot=(0.85, 1.15), strike=(85.0, 115.0), rate=(0.0, 0.06)):
    """n market points around opt: spots scaled per asset by U[spot], strikes U[strike], rates
    U[rate]. Returns (S0 [n, d], K [n], r [n]) as numpy arrays."""
    rng = _rng(seed)
    d = opt["d"]
    S0 = np.asarray(opt["S0"])[None, :] * rng.uniform(spot[0], spot[1], (n, d))
    return S0, rng.uniform(strike[0], strike[1], n), rng.uniform(rate[0], rate[1], n)
