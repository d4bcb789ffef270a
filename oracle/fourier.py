"""Fourier price of a European option on d correlated GBM assets on a truncated grid.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What is computed (paper: Sec. II.A market model, Sec. III.B Eq. maincont,
Sec. III.C Eq. main, Sec. III.D Eq. discr and the nested multi-asset sum):

* Log-moneyness x_j = ln(S_T^j / K) is Gaussian with mean
  m_j = ln(S0_j/K) + (r - sigma_j^2/2) T and covariance C = T diag(sigma) R diag(sigma)
  (the multi-asset characteristic function of Sec. III.C with the maturity T kept
  in the quadratic term).
* Max/min payoffs are split into d terms, one per asset that attains the extreme:
  (max_j e^{x_j} - 1)^+ = sum_j (e^{x_j} - 1)^+ prod_{l != j} 1{x_l < x_j}.
  In term j the coordinates are w_0 = x_j and w_l = x_l - x_j (l != j, increasing l),
  i.e. w = P_j x, so the term's payoff is a product of one-dimensional factors and
  its Gaussian has mean P_j m and covariance P_j C P_j^T. Put-on-max uses the put
  factor (1 - e^{w_0})^+; call-on-min uses 1{w_l > 0}. For d = 1 there is a single
  term with P = [1].
* Each term is a d-dimensional shifted-contour Fourier integral
  (2 pi)^{-d} int phi(-z) prod_k h_k(z_k) dz over Im z = alpha, discretised by the
  midpoint rule on [-L_k, L_k] with N nodes per coordinate; the sum itself is the
  plain loop in dense.c.
* price = K e^{-rT} Re sum_terms [prod_k (eta_k / 2 pi)] S_term.

Payoff factor transforms, derived by direct integration of int e^{i z w} f(w) dw:
  (e^w - 1)^+  -> 1/(iz(1+iz)),  Im z > 1   (equals the paper's -K^{iz+1}/(z(z-i)) at K=1)
  (1 - e^w)^+  -> 1/(iz(1+iz)),  Im z < 0
  1{w < 0}     -> 1/(iz),        Im z < 0
  1{w > 0}     -> -1/(iz),       Im z > 0

The paper's own formulation of the call on the minimum (Sec. III.C, the min transform with
Eq. main) keeps the asset coordinates and one term ("call_min_strip"): with
(min_j e^{x_j} - 1)^+ = int_0^inf e^y prod_j 1{x_j > y} dy, direct integration gives the joint
transform (-1)^(d+1) / ((1 + i sum_j z_j) prod_j (i z_j)) on Im z_j > 0, sum_j Im z_j > 1 (the
printed formula differs from this by the phase i^(d-2); at d = 1 the form here is the call
transform above).

Readings of the paper taken here: the maturity multiplies the quadratic term of the
characteristic function; the d-dimensional normalisation is (2 pi)^{-d}; the sum
uses N midpoint nodes u_i = -L + (i + 1/2) 2L/N (a symmetric grid); the bilinear
(non-conjugated) product phi(-z) v(z) is summed and its real part taken.

Grid rule (grid_rule): per term and coordinate, L_k = sqrt(2 tau (C_w^{-1})_kk)
(the marginal of exp(-u^T C_w u / 2) along u_k has variance (C_w^{-1})_kk), and the
contour shift is set from the aliasing distance X_k = 2 pi / eta_k so that
exp(-a_k X_k) = exp(-tau), with a_k the distance to the factor's pole
(alpha_0 = 1 + a_0 for a call coordinate, -a_0 for a put coordinate, -a_k / +a_k
for max / min indicators). tau = ln(100 / tol) clamped to [18, 34.5]: a tighter target
costs a larger shift, and the shift's damping e^{alpha.w} multiplies the absolute
size of the summand (the cancellation factor) faster than it removes aliasing. When the
damping exponent Phi = ln E[e^{alpha.w}] = alpha.m + alpha^T C_w alpha / 2 (plus, with Merton
jumps, lambda T (E[e^{alpha.J_w}] - 1)) of that choice exceeds 12 (coarse grids), tau is lowered by
bisection on [2, tau] (60 halvings) until Phi <= 12.

Parity: pinned in tests/test_oracle_fourier.py against Black-Scholes (d=1), the
two-asset closed forms (d=2), the one-factor quadrature (d=3, 5), put-call parity,
brute-force x-space integration of every payoff factor, and Monte Carlo.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

KIND_CALL, KIND_LT, KIND_GT, KIND_STRIP = 0, 1, 2, 3
DEFAULT_TOL = 1e-12


def grid_tau(tol):
    """Exponent of the truncation / aliasing targets for a requested tolerance."""
    return min(34.5, max(18.0, math.log(100.0 / tol)))

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        cd = ctypes.c_double
        lib.dense_term_sum.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ip, cd, dp, dp, ctypes.c_int, dp]
        lib.dense_term_sum.restype = None
        lib.dense_term_sum_rows.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ip, cd, dp, dp, ctypes.c_int,
                                            ctypes.c_int64, ctypes.c_int64, dp]
        lib.dense_term_sum_rows.restype = None
        lib.integrand_points.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ip, cd, dp, dp,
                                         ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), dp]
        lib.integrand_points.restype = None
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------------------------- model

def jumps(opt):
    """(lambda, mean[d], cov[d, d]) of the log-jump sizes of Merton's model (the extension named
    in Sec. VI); lambda = 0 when the option has no jumps."""
    d = opt["d"]
    lam = float(opt.get("jump_rate", 0.0) or 0.0)
    if lam <= 0.0:
        return 0.0, np.zeros(d), np.zeros((d, d))
    return lam, np.asarray(opt["jump_mean"], float), np.asarray(opt["jump_cov"], float)


def log_moments(opt):
    """Mean and covariance of the diffusion part of x = ln(S_T / K) under the risk-neutral
    measure: GBM, plus (with jumps) the compensator -lambda kappa_j T in the mean that keeps
    e^{-rT} S_T^j a martingale, kappa_j = E[e^{J_j}] - 1 = exp(muJ_j + CJ_jj / 2) - 1."""
    S0 = np.asarray(opt["S0"], float)
    sig = np.asarray(opt["sigma"], float)
    R = np.asarray(opt["corr"], float)
    T, r, K = opt["T"], opt["r"], opt["K"]
    m = np.log(S0 / K) + (r - 0.5 * sig ** 2) * T
    lam, muJ, CJ = jumps(opt)
    if lam > 0.0:
        m = m - lam * T * (np.exp(muJ + 0.5 * np.diag(CJ)) - 1.0)
    C = T * np.outer(sig, sig) * R
    return m, C


def terms(opt):
    """List of per-term dicts: P (rotation), m (mean of w), C (cov of w), kind[d],
    sign[d] (+1: contour above the real axis, -1: below)."""
    d = opt["d"]
    m, C = log_moments(opt)
    lam, muJ, CJ = jumps(opt)
    lamT = lam * opt["T"]
    pay = opt["payoff"]
    if pay == "call_min_strip":
        return [dict(P=np.eye(d), m=m, C=C, kind=np.full(d, KIND_STRIP, dtype=np.int32), sign=np.ones(d),
                     lamT=lamT, mJ=muJ, CJ=CJ)]
    out = []
    for j in range(d):
        P = np.zeros((d, d))
        P[0, j] = 1.0
        row = 1
        for l in range(d):
            if l == j:
                continue
            P[row, l] = 1.0
            P[row, j] = -1.0
            row += 1
        kind = np.zeros(d, dtype=np.int32)
        sign = np.zeros(d)
        kind[0] = KIND_CALL
        sign[0] = -1.0 if pay == "put_max" else 1.0
        if pay in ("call_max", "put_max"):
            kind[1:] = KIND_LT
            sign[1:] = -1.0
        elif pay == "call_min":
            kind[1:] = KIND_GT
            sign[1:] = 1.0
        else:
            raise ValueError(pay)
        out.append(dict(P=P, m=P @ m, C=P @ C @ P.T, kind=kind, sign=sign, lamT=lamT, mJ=P @ muJ, CJ=P @ CJ @ P.T))
        if d == 1:
            break
    return out


PHI_MAX = 12.0


def _rule_at(term, N, tau, prec):
    L = np.sqrt(2.0 * tau * prec)
    eta = 2.0 * L / N
    a = tau * eta / (2.0 * math.pi)
    alpha = np.empty_like(L)
    for k in range(len(L)):
        if term["kind"][k] == KIND_CALL and term["sign"][k] > 0:
            alpha[k] = 1.0 + a[k]
        elif term["kind"][k] == KIND_STRIP:
            alpha[k] = a[k] + 1.0 / len(L)       # distance a_k from z_k = 0, sum a_k from sum z = i
        else:
            alpha[k] = term["sign"][k] * a[k]
    phi = float(alpha @ term["m"] + 0.5 * alpha @ term["C"] @ alpha)
    lamT = float(term.get("lamT", 0.0))
    if lamT > 0.0:
        # the jump part of the cumulant generating function: lambda T (E[e^{alpha.J}] - 1)
        phi += lamT * math.expm1(float(alpha @ term["mJ"] + 0.5 * alpha @ term["CJ"] @ alpha))
    return L, alpha, phi


def grid_rule(term, N, tol=DEFAULT_TOL):
    """Automatic (L_k, alpha_k) for one term (see module docstring)."""
    tau = grid_tau(tol)
    prec = np.diag(np.linalg.inv(term["C"]))
    L, alpha, phi = _rule_at(term, N, tau, prec)
    if phi > PHI_MAX:
        lo, hi = 2.0, tau
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if _rule_at(term, N, mid, prec)[2] <= PHI_MAX:
                lo = mid
            else:
                hi = mid
        L, alpha, phi = _rule_at(term, N, lo, prec)
    return L, alpha


def term_grids(opt, N, L=None, alpha=None, tol=DEFAULT_TOL):
    """Per-term (L[d], alpha[d]) arrays. L/alpha may be None (automatic rule),
    a positive scalar (same half-width / same |shift| on every coordinate, with the
    sign of each coordinate's strip; a call coordinate takes +alpha), or an array of
    shape [n_terms, d] taken as given."""
    ts = terms(opt)
    out = []
    for t, term in enumerate(ts):
        Lauto, Aauto = grid_rule(term, N, tol)
        if L is None:
            Lt = Lauto
        elif np.isscalar(L):
            Lt = np.full(opt["d"], float(L))
        else:
            Lt = np.asarray(L, float)[t]
        if alpha is None:
            if L is None:
                At = Aauto
            else:   # rule for alpha given this L
                eta = 2.0 * Lt / N
                a = grid_tau(tol) * eta / (2.0 * math.pi)
                At = np.where((term["kind"] == KIND_CALL) & (term["sign"] > 0), 1.0 + a, term["sign"] * a)
                At = np.where(term["kind"] == KIND_STRIP, a + 1.0 / opt["d"], At)
        elif np.isscalar(alpha):
            At = term["sign"] * float(alpha)
        else:
            At = np.asarray(alpha, float)[t]
        out.append((np.ascontiguousarray(Lt, float), np.ascontiguousarray(At, float)))
    return ts, out


def _jump_args(term, d):
    lamT = float(term.get("lamT", 0.0))
    mJ = np.ascontiguousarray(term.get("mJ", np.zeros(d)), float)
    CJ = np.ascontiguousarray(term.get("CJ", np.zeros((d, d))), float)
    return lamT, mJ, CJ


def dense_term(term, N, L, alpha, nthreads=0):
    """(complex S, sum |F|) for one term."""
    lib = _load()
    d = len(term["m"])
    m = np.ascontiguousarray(term["m"], float)
    C = np.ascontiguousarray(term["C"], float)
    kind = np.ascontiguousarray(term["kind"], np.int32)
    L = np.ascontiguousarray(L, float)
    alpha = np.ascontiguousarray(alpha, float)
    lamT, mJ, CJ = _jump_args(term, d)
    out = np.zeros(3)
    lib.dense_term_sum(d, N, _dp(m), _dp(C), _dp(L), _dp(alpha),
                       kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), lamT, _dp(mJ), _dp(CJ), int(nthreads),
                       _dp(out))
    return complex(out[0], out[1]), float(out[2])


def dense_term_rows(term, N, L, alpha, row_begin, row_end, nthreads=0):
    """Partial dense sum over grid rows [row_begin, row_end) (a row fixes all but the last index)."""
    lib = _load()
    d = len(term["m"])
    m = np.ascontiguousarray(term["m"], float)
    C = np.ascontiguousarray(term["C"], float)
    kind = np.ascontiguousarray(term["kind"], np.int32)
    L = np.ascontiguousarray(L, float)
    alpha = np.ascontiguousarray(alpha, float)
    lamT, mJ, CJ = _jump_args(term, d)
    out = np.zeros(3)
    lib.dense_term_sum_rows(d, N, _dp(m), _dp(C), _dp(L), _dp(alpha),
                            kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), lamT, _dp(mJ), _dp(CJ), int(nthreads),
                            int(row_begin), int(row_end), _dp(out))
    return complex(out[0], out[1]), float(out[2])


def term_scale(opt, L, N):
    """K e^{-rT} prod_k (eta_k / 2 pi) for one term with half-widths L."""
    eta = 2.0 * np.asarray(L, float) / N
    return opt["K"] * math.exp(-opt["r"] * opt["T"]) * float(np.prod(eta / (2.0 * math.pi)))


def dense_price(opt, N, L=None, alpha=None, nthreads=0, details=False, tol=DEFAULT_TOL):
    """The Fourier price on the full N^d grid of every term (tol selects the automatic grid)."""
    ts, grids = term_grids(opt, N, L, alpha, tol)
    total = 0.0 + 0.0j
    abs_total = 0.0
    per_term = []
    for term, (Lt, At) in zip(ts, grids):
        s, sa = dense_term(term, N, Lt, At, nthreads)
        sc = term_scale(opt, Lt, N)
        per_term.append(sc * s)
        total += sc * s
        abs_total += sc * sa
    if details:
        return dict(price=total.real, imag=total.imag, terms=per_term, abs_sum=abs_total,
                    kappa=abs_total / abs(total.real) if total.real != 0 else float("inf"),
                    grids=grids)
    return total.real


def integrand_at(term, N, L, alpha, idx):
    """Integrand values (complex) of one term at integer multi-indices idx[n, d]."""
    lib = _load()
    d = len(term["m"])
    idx = np.ascontiguousarray(idx, np.int32)
    n = idx.shape[0]
    out = np.zeros(2 * n)
    m = np.ascontiguousarray(term["m"], float)
    C = np.ascontiguousarray(term["C"], float)
    kind = np.ascontiguousarray(term["kind"], np.int32)
    L = np.ascontiguousarray(L, float)
    alpha = np.ascontiguousarray(alpha, float)
    lamT, mJ, CJ = _jump_args(term, d)
    lib.integrand_points(d, N, _dp(m), _dp(C), _dp(L), _dp(alpha),
                         kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), lamT, _dp(mJ), _dp(CJ), n,
                         idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(out))
    return out[0::2] + 1j * out[1::2]


def payoff_factor(kind, z):
    """Transform of one payoff factor (kind as in dense.c), NumPy version for tests."""
    z = np.asarray(z, complex)
    iz = 1j * z
    if kind == KIND_CALL:
        return 1.0 / (iz * (1.0 + iz))
    if kind == KIND_LT:
        return 1.0 / iz
    return -1.0 / iz


def min_strip_transform(z):
    """Joint transform of (min_j e^{w_j} - 1)^+ (K = 1) at complex z[d] with Im z_j > 0 and
    sum_j Im z_j > 1: (-1)^(d+1) / ((1 + i sum z) prod (i z_j)) (NumPy version for tests)."""
    z = np.asarray(z, complex)
    d = z.shape[-1]
    return (-1.0) ** (d + 1) / ((1.0 + 1j * z.sum(axis=-1)) * np.prod(1j * z, axis=-1))


def paper_min_transform(z, K=1.0):
    """The d-dimensional call-on-min transform exactly as printed in Sec. III.C
    (kept only so that a test can show it disagrees with the one-asset transform)."""
    z = np.asarray(z, complex)
    s = np.sum(z)
    d = len(z)
    return K ** (1 + 1j * s) / ((-1) ** d * (1 + 1j * s) * np.prod(z))
