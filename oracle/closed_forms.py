"""Closed forms and semi-closed forms used to pin the Fourier oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Black-Scholes call/put and their delta and vega: the exact single-asset solution
  (Sec. II, Eq. BSexact), with d_{1,2} as defined there.
* bivariate_normal_cdf: P(X <= a, Y <= b) for standard normals with correlation rho,
  computed from its definition as a one-dimensional integral of the conditional CDF.
* stulz_call_min / stulz_call_max: two-asset call on the minimum / maximum under
  correlated GBM (Sec. II.A market model). Derived by changes of numeraire: each
  "asset j is the extreme one and finishes in the money" event is a bivariate
  normal probability under the measure that uses asset j as numeraire.
* margrabe_exchange: value of the option to exchange asset 2 for asset 1.
* one_factor_price: call/put on max/min of d assets when the correlation is
  rho 1 1^T + (1 - rho) I with rho >= 0 (this contains the paper's family
  Sigma(beta), Sec. V.B Eq. covmat). Conditional on the common factor the assets
  are independent, so P(max S_T <= s) is an expectation of a product of normal
  CDFs; the price is the integral of the tail probability over the strike axis.

Parity: every function here is pinned by an independent route in
tests/test_oracle_closed_forms.py (special cases, a second formula, brute force).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def norm_cdf(x):
    return special.ndtr(x)


def norm_pdf(x):
    return np.exp(-0.5 * np.asarray(x, dtype=float) ** 2) / math.sqrt(2.0 * math.pi)


# ------------------------------------------------------------------ Black-Scholes (Eq. BSexact)

def _d12(S0, K, T, r, sigma):
    v = sigma * math.sqrt(T)
    d1 = (math.log(S0 / K) + (r + 0.5 * sigma * sigma) * T) / v
    return d1, d1 - v


def bs_call(S0, K, T, r, sigma):
    d1, d2 = _d12(S0, K, T, r, sigma)
    return S0 * norm_cdf(d1) - K * math.exp(-r * T) * norm_cdf(d2)


def bs_put(S0, K, T, r, sigma):
    d1, d2 = _d12(S0, K, T, r, sigma)
    return K * math.exp(-r * T) * norm_cdf(-d2) - S0 * norm_cdf(-d1)


def bs_call_delta(S0, K, T, r, sigma):
    return float(norm_cdf(_d12(S0, K, T, r, sigma)[0]))


def bs_vega(S0, K, T, r, sigma):
    d1, _ = _d12(S0, K, T, r, sigma)
    return float(S0 * norm_pdf(d1) * math.sqrt(T))


# ------------------------------------------------------------------ bivariate normal

def bivariate_normal_cdf(a, b, rho):
    """P(X <= a, Y <= b), (X, Y) standard normal with correlation rho, as
    int_{-inf}^{a} phi(x) Phi((b - rho x) / sqrt(1 - rho^2)) dx."""
    if rho >= 1.0:
        return float(norm_cdf(min(a, b)))
    if rho <= -1.0:
        return float(max(0.0, norm_cdf(a) - norm_cdf(-b)))
    s = math.sqrt(1.0 - rho * rho)

    def f(x):
        return math.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi) * norm_cdf((b - rho * x) / s)

    lo = -40.0
    if a <= lo:
        return 0.0
    # split at 0 and at the kink region so that quad sees smooth pieces
    pts = sorted({p for p in (0.0, b / rho if rho != 0 else 0.0) if lo < p < a})
    edges = [lo] + pts + [a]
    total = 0.0
    for x0, x1 in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(f, x0, x1, epsabs=1e-17, epsrel=1e-14, limit=400)
        total += val
    return total


# ------------------------------------------------------------------ two-asset closed forms

def stulz_call_min(S1, S2, K, T, r, s1, s2, rho):
    """Call on min(S1_T, S2_T) with strike K (two-asset closed form)."""
    sq = math.sqrt(T)
    g1 = (math.log(S1 / K) + (r - 0.5 * s1 * s1) * T) / (s1 * sq)
    g2 = (math.log(S2 / K) + (r - 0.5 * s2 * s2) * T) / (s2 * sq)
    sb = math.sqrt(s1 * s1 + s2 * s2 - 2.0 * rho * s1 * s2)
    a1 = (math.log(S2 / S1) - 0.5 * sb * sb * T) / (sb * sq)
    a2 = (math.log(S1 / S2) - 0.5 * sb * sb * T) / (sb * sq)
    t1 = S1 * bivariate_normal_cdf(g1 + s1 * sq, a1, (rho * s2 - s1) / sb)
    t2 = S2 * bivariate_normal_cdf(g2 + s2 * sq, a2, (rho * s1 - s2) / sb)
    t3 = K * math.exp(-r * T) * bivariate_normal_cdf(g1, g2, rho)
    return t1 + t2 - t3


def stulz_call_max(S1, S2, K, T, r, s1, s2, rho):
    """Call on max = BS call on 1 + BS call on 2 - call on min."""
    return (bs_call(S1, K, T, r, s1) + bs_call(S2, K, T, r, s2)
            - stulz_call_min(S1, S2, K, T, r, s1, s2, rho))


def margrabe_exchange(S1, S2, T, s1, s2, rho):
    """Value of max(S1_T - S2_T, 0) (discounted), the exchange option."""
    sb = math.sqrt(s1 * s1 + s2 * s2 - 2.0 * rho * s1 * s2)
    d1 = (math.log(S1 / S2) + 0.5 * sb * sb * T) / (sb * math.sqrt(T))
    d2 = d1 - sb * math.sqrt(T)
    return S1 * norm_cdf(d1) - S2 * norm_cdf(d2)


def discounted_expected_max2(S1, S2, T, s1, s2, rho):
    """e^{-rT} E[max(S1_T, S2_T)] = S2 + exchange value (independent of r)."""
    return S2 + margrabe_exchange(S1, S2, T, s1, s2, rho)


# ------------------------------------------------------------------ Merton jumps: series over the jump count

def merton_series(S0, K, T, r, sigma, corr, lam, muJ, CJ, payoff="call_max", n_max=None):
    """Price under Merton's jump diffusion (the extension of Sec. VI) with log-jump sizes
    N(muJ, CJ) arriving at rate lam (one Poisson clock for all assets), d = 1 or 2, by
    conditioning on the number n of jumps: given n, ln(S_T) is Gaussian with mean
    ln S0 + (r - sigma^2/2 - lam kappa) T + n muJ and covariance T diag(sigma) corr diag(sigma)
    + n CJ (kappa_j = exp(muJ_j + CJ_jj / 2) - 1), which is a GBM with adjusted spots, volatilities
    and correlation: priced by Black-Scholes (d = 1) or Stulz (d = 2), weighted by the Poisson
    probabilities."""
    S0 = np.atleast_1d(np.asarray(S0, float))
    sigma = np.atleast_1d(np.asarray(sigma, float))
    d = len(S0)
    corr = np.asarray(corr, float).reshape(d, d)
    muJ = np.atleast_1d(np.asarray(muJ, float))
    CJ = np.asarray(CJ, float).reshape(d, d)
    kappa = np.exp(muJ + 0.5 * np.diag(CJ)) - 1.0
    C0 = T * np.outer(sigma, sigma) * corr
    lt = lam * T
    if n_max is None:
        n_max = int(lt + 12.0 * math.sqrt(lt + 1.0) + 20)
    total = 0.0
    for n in range(n_max + 1):
        w = math.exp(-lt + n * math.log(lt) - math.lgamma(n + 1)) if lt > 0 else (1.0 if n == 0 else 0.0)
        if w == 0.0:
            continue
        C = C0 + n * CJ
        s = np.sqrt(np.diag(C) / T)
        # forward of asset j given n jumps: S0 e^{(r - lam kappa) T + n (muJ + CJ_jj / 2)}
        fwd = S0 * np.exp((r - lam * kappa) * T + n * (muJ + 0.5 * np.diag(CJ)))
        S_eff = fwd * math.exp(-r * T)
        if d == 1:
            v = bs_call(S_eff[0], K, T, r, s[0])
        elif payoff == "call_max":
            v = stulz_call_max(S_eff[0], S_eff[1], K, T, r, s[0], s[1], C[0, 1] / (T * s[0] * s[1]))
        elif payoff == "call_min":
            v = stulz_call_min(S_eff[0], S_eff[1], K, T, r, s[0], s[1], C[0, 1] / (T * s[0] * s[1]))
        else:
            raise ValueError(payoff)
        total += w * v
    return total


# ------------------------------------------------------------------ one-factor quadrature, any d

def one_factor_price(S0, K, T, r, sigma, rho, payoff="call_max", n_hermite=160):
    """Price of a call/put on the max/min of d GBM assets whose correlation matrix
    is rho on every off-diagonal entry (rho >= 0).

    X_j = ln S_T^j = mu_j + sigma_j sqrt(T) (sqrt(rho) M + sqrt(1-rho) Z_j),
    mu_j = ln S0_j + (r - sigma_j^2/2) T, with M, Z_j independent standard normals.
    Given M the X_j are independent, so with z_j(y) = (y - mu_j - b_j M)/c_j,
    b_j = sigma_j sqrt(rho T), c_j = sigma_j sqrt((1-rho) T):
        P(max_j X_j <= y | M) = prod_j Phi(z_j),   P(min_j X_j > y | M) = prod_j Phi(-z_j).
    call_max = e^{-rT} int_{ln K}^{inf} e^y (1 - E_M prod Phi(z_j)) dy
    call_min = e^{-rT} int_{ln K}^{inf} e^y E_M prod Phi(-z_j) dy
    put_max  = e^{-rT} int_{-inf}^{ln K} e^y E_M prod Phi(z_j) dy
    E_M is taken by Gauss-Hermite quadrature (probabilists' weight), the y integral
    adaptively.
    """
    S0 = np.asarray(S0, float)
    sigma = np.asarray(sigma, float)
    if not (0.0 <= rho < 1.0):
        raise ValueError("one-factor form needs 0 <= rho < 1")
    mu = np.log(S0) + (r - 0.5 * sigma ** 2) * T
    b = sigma * math.sqrt(rho * T)
    c = sigma * math.sqrt((1.0 - rho) * T)
    xm, wm = np.polynomial.hermite_e.hermegauss(n_hermite)
    wm = wm / math.sqrt(2.0 * math.pi)
    lnK = math.log(K)
    spread = 14.0 * float(np.max(sigma)) * math.sqrt(T)

    def zmat(y):
        return (y - mu[None, :] - b[None, :] * xm[:, None]) / c[None, :]

    if payoff == "call_max":
        def f(y):
            # 1 - prod Phi(z) = -expm1(sum log1p(-Phi(-z)))
            q = special.ndtr(-zmat(y))
            tail = -np.expm1(np.sum(np.log1p(-q), axis=1))
            return math.exp(y) * float(np.dot(wm, tail))
        lo, hi = lnK, max(lnK, float(np.max(mu))) + spread
    elif payoff == "call_min":
        def f(y):
            p = np.prod(special.ndtr(-zmat(y)), axis=1)
            return math.exp(y) * float(np.dot(wm, p))
        lo, hi = lnK, max(lnK, float(np.max(mu))) + spread
    elif payoff == "put_max":
        def f(y):
            p = np.prod(special.ndtr(zmat(y)), axis=1)
            return math.exp(y) * float(np.dot(wm, p))
        lo, hi = min(lnK, float(np.min(mu))) - spread, lnK
    else:
        raise ValueError(payoff)
    if hi <= lo:
        return 0.0
    edges = np.linspace(lo, hi, 17)
    total = 0.0
    for y0, y1 in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(f, y0, y1, epsabs=1e-15 * K, epsrel=1e-14, limit=400)
        total += v
    return math.exp(-r * T) * total
