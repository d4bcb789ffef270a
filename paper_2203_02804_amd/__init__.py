"""Tensor-train Fourier pricing of multi-asset options on AMD MI355X.

Thin Python binding over the C ABI in include/ttfp.h (libttfp.so, built by
paper_2203_02804_amd/build.py). Only argument marshalling happens here: every step of
the pricing path runs in the library's HIP kernels. PyTorch is used for the device
choice and the HIP stream the library enqueues on.

Options and grids are the dicts produced by the `workloads` module:
    option: d, S0, K, T, r, sigma, corr, payoff ("call_max" | "put_max" | "call_min")
    grid:   N, L, alpha, tol, max_rank, max_sweeps, seed (+ optional n_enrich, rank_tol)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttfp.so")

PAYOFF_CODES = {"call_max": 0, "put_max": 1, "call_min": 2, "call_min_strip": 3}
TTFP_OK, TTFP_EINVAL, TTFP_ENOMEM, TTFP_EDEVICE, TTFP_ENOTCONV, TTFP_EPRECISION = 0, -1, -2, -3, 1, 2
MAX_RANK = 64


class TTFPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ttfp error {code}: {msg}")
        self.code = code


class _Option(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("payoff", ctypes.c_int32),
                ("S0", ctypes.POINTER(ctypes.c_double)), ("sigma", ctypes.POINTER(ctypes.c_double)),
                ("corr", ctypes.POINTER(ctypes.c_double)),
                ("K", ctypes.c_double), ("T", ctypes.c_double), ("r", ctypes.c_double),
                ("jump_rate", ctypes.c_double), ("jump_mean", ctypes.POINTER(ctypes.c_double)),
                ("jump_cov", ctypes.POINTER(ctypes.c_double))]


class _Grid(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("L", ctypes.c_double), ("alpha", ctypes.c_double),
                ("L_k", ctypes.POINTER(ctypes.c_double)), ("alpha_k", ctypes.POINTER(ctypes.c_double)),
                ("tol", ctypes.c_double), ("rank_tol", ctypes.c_double),
                ("max_rank", ctypes.c_int32), ("max_sweeps", ctypes.c_int32), ("n_enrich", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("n_err_samples", ctypes.c_int32),
                ("certify", ctypes.c_int32)]


class _Diag(ctypes.Structure):
    _fields_ = [("imag_rel", ctypes.c_double), ("kappa", ctypes.c_double), ("last_change", ctypes.c_double),
                ("n_evals", ctypes.c_int64), ("maxvol_swaps", ctypes.c_int64),
                ("sweeps", ctypes.c_int32), ("rank_capped", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("maxvol_full_starts", ctypes.c_int64), ("err_est", ctypes.c_double), ("err_samples", ctypes.c_int64)]


EXPORTS = ["ttfp_create", "ttfp_destroy", "ttfp_plan", "ttfp_price", "ttfp_price_batch", "ttfp_batch_diag", "ttfp_price_batch_noalloc", "ttfp_price_ladder", "ttfp_price_two_trains", "ttfp_eval_integrand",
           "ttfp_tt_values", "ttfp_tt_export", "ttfp_qr_r", "ttfp_maxvol", "ttfp_strerror", "ttfp_last_error",
           "ttfp_profile_enable", "ttfp_profile_read", "ttfp_set_tuning", "ttfp_get_tuning", "ttfp_mlp_create", "ttfp_mlp_destroy", "ttfp_mlp_n_params",
           "ttfp_mlp_get_params", "ttfp_mlp_set_params", "ttfp_mlp_forward", "ttfp_mlp_grad", "ttfp_mlp_train_step",
           "ttfp_mlp_last_error"]
KERNELS = ["fiber", "tsqr", "qrcp", "basis", "maxvol", "finish", "core_sum", "contract", "interp", "err_est",
           "gram", "chol", "xform", "ladder", "refine"]
TUNING = {"maxvol_rounds": 0, "tsqr_lds_kb": 1, "graph": 2, "qr": 3, "maxvol_warm": 4, "mm_waves": 5, "gram_threads": 6, "mm_panels": 7, "interp_bound": 8}

_lib = None


def load():
    """Loads libttfp.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2203_02804_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.ttfp_create.argtypes = [P(vp), ctypes.c_int, vp]
    lib.ttfp_destroy.argtypes = [vp]
    lib.ttfp_plan.argtypes = [P(_Option), P(_Grid), P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double)]
    lib.ttfp_price.argtypes = [vp, P(_Option), P(_Grid), P(ctypes.c_double), P(ctypes.c_int32), P(_Diag)]
    lib.ttfp_price_batch.argtypes = [vp, ctypes.c_int32, P(_Option), P(_Grid), P(ctypes.c_double),
                                     P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_int32)]
    lib.ttfp_price_batch_noalloc.argtypes = lib.ttfp_price_batch.argtypes
    lib.ttfp_price_two_trains.argtypes = [vp, P(_Option), P(_Grid), ctypes.c_int32, P(ctypes.c_double),
                                          P(ctypes.c_int32), P(ctypes.c_int32), P(_Diag)]
    lib.ttfp_price_ladder.argtypes = [vp, P(_Option), P(_Grid), ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double),
                                      P(ctypes.c_double), P(ctypes.c_double), P(_Diag)]
    lib.ttfp_batch_diag.argtypes = [vp, ctypes.c_int32, P(_Diag)]
    lib.ttfp_eval_integrand.argtypes = [vp, P(_Option), P(_Grid), ctypes.c_int32, ctypes.c_int64,
                                        P(ctypes.c_int32), P(ctypes.c_double)]
    lib.ttfp_tt_values.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, P(ctypes.c_int32), P(ctypes.c_double)]
    lib.ttfp_tt_export.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_int32),
                                   P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.ttfp_qr_r.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double)]
    lib.ttfp_maxvol.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double), ctypes.c_double,
                                P(ctypes.c_int32), P(ctypes.c_double)]
    lib.ttfp_profile_enable.argtypes = [vp, ctypes.c_int]
    lib.ttfp_profile_read.argtypes = [vp, ctypes.c_int, P(ctypes.c_int64), P(ctypes.c_double), P(ctypes.c_double)]
    lib.ttfp_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.ttfp_get_tuning.argtypes = [vp, ctypes.c_int, P(ctypes.c_int)]
    lib.ttfp_strerror.argtypes = [ctypes.c_int]
    lib.ttfp_strerror.restype = ctypes.c_char_p
    lib.ttfp_last_error.argtypes = [vp]
    lib.ttfp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class _Marshal:
    """Keeps the numpy arrays behind a ctypes option/grid alive."""

    def __init__(self, opt, grid):
        d = int(opt["d"])
        self.S0 = np.ascontiguousarray(opt["S0"], np.float64)
        self.sigma = np.ascontiguousarray(opt["sigma"], np.float64)
        self.corr = np.ascontiguousarray(opt["corr"], np.float64).reshape(-1)
        if self.S0.shape != (d,) or self.sigma.shape != (d,) or self.corr.shape != (d * d,):
            raise ValueError("option arrays do not match d")
        lam = float(opt.get("jump_rate", 0.0) or 0.0)
        null = ctypes.POINTER(ctypes.c_double)()
        self.jm = self.jc = None
        if lam > 0.0:
            self.jm = np.ascontiguousarray(opt["jump_mean"], np.float64).reshape(-1)
            self.jc = np.ascontiguousarray(opt["jump_cov"], np.float64).reshape(-1)
            if self.jm.shape != (d,) or self.jc.shape != (d * d,):
                raise ValueError("jump arrays do not match d")
        self.opt = _Option(d, PAYOFF_CODES[opt.get("payoff", "call_max")], _dp(self.S0), _dp(self.sigma),
                           _dp(self.corr), float(opt["K"]), float(opt["T"]), float(opt["r"]), lam,
                           _dp(self.jm) if self.jm is not None else null, _dp(self.jc) if self.jc is not None else null)
        L, A = grid.get("L"), grid.get("alpha")
        self.Lk = self.Ak = None
        Ls = As = 0.0
        if L is not None and np.ndim(L) == 0:
            Ls = float(L)
        elif L is not None:
            self.Lk = np.ascontiguousarray(L, np.float64).reshape(-1)
        if A is not None and np.ndim(A) == 0:
            As = float(A)
        elif A is not None:
            self.Ak = np.ascontiguousarray(A, np.float64).reshape(-1)
        null = ctypes.POINTER(ctypes.c_double)()
        self.grid = _Grid(int(grid["N"]), Ls, As,
                          _dp(self.Lk) if self.Lk is not None else null,
                          _dp(self.Ak) if self.Ak is not None else null,
                          float(grid.get("tol", 1e-8)), float(grid.get("rank_tol", 0.0)),
                          int(grid.get("max_rank", 32)), int(grid.get("max_sweeps", 6)),
                          int(grid.get("n_enrich", 4)), int(grid.get("seed", 0)) & ((1 << 64) - 1),
                          int(grid.get("n_err_samples", 0)), int(grid.get("certify", 0)))


def plan(opt, grid):
    """Per-term (L, alpha) arrays [n_terms, d] the pricer uses (host logic, no device)."""
    lib = load()
    m = _Marshal(opt, grid)
    d = int(opt["d"])
    nt = ctypes.c_int32(0)
    L = np.zeros(d * d)
    A = np.zeros(d * d)
    rc = lib.ttfp_plan(ctypes.byref(m.opt), ctypes.byref(m.grid), ctypes.byref(nt), _dp(L), _dp(A))
    if rc < 0:
        raise TTFPError(rc, lib.ttfp_strerror(rc).decode())
    n = nt.value
    return L[: n * d].reshape(n, d), A[: n * d].reshape(n, d)


def _diag_dict(diag):
    return dict(imag_rel=diag.imag_rel, kappa=diag.kappa, last_change=diag.last_change, n_evals=diag.n_evals,
                maxvol_swaps=diag.maxvol_swaps, maxvol_full_starts=diag.maxvol_full_starts,
                sweeps=diag.sweeps, rank_capped=bool(diag.rank_capped), converged=bool(diag.converged),
                err_est=diag.err_est, err_samples=diag.err_samples)


class Pricer:
    """A library context bound to one HIP device and stream."""

    def __init__(self, device=0, stream=None):
        import torch

        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.ctx = ctypes.c_void_p()
        rc = self.lib.ttfp_create(ctypes.byref(self.ctx), int(device), ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise TTFPError(rc, "ttfp_create failed")
        # price_batch applies the autotuner's stored launch setting for its batch's shape (only
        # settings that leave results unchanged bit for bit); False keeps the context's own
        self.autotune = True

    def _apply_tuned(self, opts, grids):
        if not self.autotune or not opts:
            return None
        ds = {int(o["d"]) for o in opts}
        Ns = {int(g["N"]) for g in grids}
        Rs = {int(g.get("max_rank", 32)) for g in grids}
        if len(ds) == 1 and len(Ns) == 1 and len(Rs) == 1:
            from . import tuning
            return tuning.apply(self, ds.pop(), Ns.pop(), Rs.pop())
        return None

    def close(self):
        if self.ctx:
            self.lib.ttfp_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise TTFPError(rc, self.lib.ttfp_last_error(self.ctx).decode())
        return rc

    def price(self, opt, grid):
        """Returns (price, ranks[n_terms, d+1], diag dict, return code); n_terms is d for the
        max/min payoffs (one term per asset, 1 when d = 1) and 1 for call_min_strip."""
        m = _Marshal(opt, grid)
        d = int(opt["d"])
        out = ctypes.c_double(0.0)
        ranks = np.zeros(d * (d + 1), np.int32)
        diag = _Diag()
        rc = self._check(self.lib.ttfp_price(self.ctx, ctypes.byref(m.opt), ctypes.byref(m.grid), ctypes.byref(out),
                                             _ip(ranks), ctypes.byref(diag)))
        n_terms = 1 if (d == 1 or opt.get("payoff") == "call_min_strip") else d
        return out.value, ranks[: n_terms * (d + 1)].reshape(n_terms, d + 1), _diag_dict(diag), rc

    def price_two_trains(self, opt, grid, payoff_rank=0):
        """The two-train variant (ttfp_price_two_trains): returns (price, ranks of the
        characteristic-function trains [n_terms, d+1], ranks of the payoff trains, diag, code)."""
        m = _Marshal(opt, grid)
        d = int(opt["d"])
        out = ctypes.c_double(0.0)
        rcf = np.zeros(d * (d + 1), np.int32)
        rpy = np.zeros(d * (d + 1), np.int32)
        diag = _Diag()
        rc = self._check(self.lib.ttfp_price_two_trains(self.ctx, ctypes.byref(m.opt), ctypes.byref(m.grid),
                                                        int(payoff_rank), ctypes.byref(out), _ip(rcf), _ip(rpy),
                                                        ctypes.byref(diag)))
        n_terms = 1 if (d == 1 or opt.get("payoff") == "call_min_strip") else d
        shape = (n_terms, d + 1)
        return out.value, rcf[: n_terms * (d + 1)].reshape(shape), rpy[: n_terms * (d + 1)].reshape(shape), \
            _diag_dict(diag), rc

    def price_ladder(self, opt, grid, S0_points, K_points, r_points):
        """Prices of opt at a ladder of market points (spots S0_points [n, d], strikes K_points [n],
        rates r_points [n]) from one cross of opt (see ttfp_price_ladder). Returns (prices [n],
        diag dict of the base cross, return code)."""
        m = _Marshal(opt, grid)
        d = int(opt["d"])
        S0p = np.ascontiguousarray(S0_points, np.float64).reshape(-1, d)
        n = S0p.shape[0]
        Kp = np.ascontiguousarray(K_points, np.float64).reshape(n)
        rp = np.ascontiguousarray(r_points, np.float64).reshape(n)
        out = np.zeros(n)
        diag = _Diag()
        rc = self._check(self.lib.ttfp_price_ladder(self.ctx, ctypes.byref(m.opt), ctypes.byref(m.grid), n, _dp(S0p),
                                                    _dp(Kp), _dp(rp), _dp(out), ctypes.byref(diag)))
        return out, _diag_dict(diag), rc

    def batch_diag(self, i):
        """Diagnostics dict of option i of the last price_batch call."""
        diag = _Diag()
        self._check(self.lib.ttfp_batch_diag(self.ctx, int(i), ctypes.byref(diag)))
        return _diag_dict(diag)

    def price_batch(self, opts, grids, greeks=False, noalloc=False):
        """Prices a list of options in one batched pass. grids: one dict or a list.
        Returns prices[n] (and delta, vega lists of per-option arrays when greeks=True), status[n].
        noalloc=True calls the allocation-free entry point (workspace in the library's static
        per-GPU scratch array; batches that do not fit raise TTFPError with TTFP_EINVAL)."""
        n = len(opts)
        if isinstance(grids, dict):
            grids = [grids] * n
        self._apply_tuned(opts, grids)
        ms = [_Marshal(o, g) for o, g in zip(opts, grids)]
        copts = (_Option * n)(*[m.opt for m in ms])
        cgrids = (_Grid * n)(*[m.grid for m in ms])
        prices = np.zeros(n)
        status = np.zeros(n, np.int32)
        tot = sum(int(o["d"]) for o in opts)
        delta = np.zeros(tot) if greeks else None
        vega = np.zeros(tot) if greeks else None
        null = ctypes.POINTER(ctypes.c_double)()
        fn = self.lib.ttfp_price_batch_noalloc if noalloc else self.lib.ttfp_price_batch
        self._check(fn(self.ctx, n, copts, cgrids, _dp(prices), _dp(delta) if greeks else null,
                       _dp(vega) if greeks else null, _ip(status)))
        if not greeks:
            return prices, status
        split = np.cumsum([int(o["d"]) for o in opts])[:-1]
        return prices, np.split(delta, split), np.split(vega, split), status

    def set_tuning(self, **kw):
        """set_tuning(maxvol_rounds=..., tsqr_lds_kb=..., graph=..., qr=...)"""
        for k, v in kw.items():
            self._check(self.lib.ttfp_set_tuning(self.ctx, TUNING[k], int(v)))

    def get_tuning(self):
        out = {}
        for k, code in TUNING.items():
            v = ctypes.c_int(0)
            self._check(self.lib.ttfp_get_tuning(self.ctx, code, ctypes.byref(v)))
            out[k] = v.value
        return out

    def profile(self, enable=True):
        """Starts (and resets) or stops per-kernel device timing with HIP events."""
        self._check(self.lib.ttfp_profile_enable(self.ctx, 1 if enable else 0))

    def profile_read(self):
        """{kernel: (launches, total_ms, work)} since the last profile(True); work is bytes
        (fiber) or FP64 flops (tsqr, basis, maxvol)."""
        out = {}
        for k, name in enumerate(KERNELS):
            n = ctypes.c_int64(0)
            ms = ctypes.c_double(0.0)
            w = ctypes.c_double(0.0)
            self._check(self.lib.ttfp_profile_read(self.ctx, k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(w)))
            out[name] = (n.value, ms.value, w.value)
        return out

    def eval_integrand(self, opt, grid, term, idx):
        m = _Marshal(opt, grid)
        idx = np.ascontiguousarray(idx, np.int32)
        out = np.zeros(2 * idx.shape[0])
        self._check(self.lib.ttfp_eval_integrand(self.ctx, ctypes.byref(m.opt), ctypes.byref(m.grid), int(term),
                                                 idx.shape[0], _ip(idx), _dp(out)))
        return out[0::2] + 1j * out[1::2]

    def tt_values(self, term, idx):
        idx = np.ascontiguousarray(idx, np.int32)
        out = np.zeros(2 * idx.shape[0])
        self._check(self.lib.ttfp_tt_values(self.ctx, int(term), idx.shape[0], _ip(idx), _dp(out)))
        return out[0::2] + 1j * out[1::2]

    def tt_export(self, term, d, max_rank, N):
        """Tensor train and final index sets of term `term` of the last price() call:
        dict(ranks, cores[k] (r_k, N, r_k+1), I[k] (|I_k|, k), J[k] (|J_k|, d-k))."""
        ranks = np.zeros(d + 1, np.int32)
        sizes = np.zeros(2 * (d + 1), np.int32)
        left = np.zeros((d + 1) * max_rank * d, np.int32)
        right = np.zeros((d + 1) * max_rank * d, np.int32)
        self._check(self.lib.ttfp_tt_export(self.ctx, int(term), _ip(ranks), None, _ip(sizes), _ip(left), _ip(right)))
        total = sum(int(ranks[k]) * N * int(ranks[k + 1]) for k in range(d))
        buf = np.zeros(2 * total)
        self._check(self.lib.ttfp_tt_export(self.ctx, int(term), _ip(ranks), _dp(buf), None, None, None))
        z = buf[0::2] + 1j * buf[1::2]
        cores, off = [], 0
        for k in range(d):
            n = int(ranks[k]) * N * int(ranks[k + 1])
            cores.append(z[off:off + n].reshape(int(ranks[k]), N, int(ranks[k + 1])))
            off += n
        left = left.reshape(d + 1, max_rank, d)
        right = right.reshape(d + 1, max_rank, d)
        I = [left[k, :sizes[k], :k].copy() for k in range(d + 1)]
        J = [right[k, :sizes[d + 1 + k], k:].copy() for k in range(d + 1)]
        return dict(ranks=ranks, cores=cores, I=I, J=J)

    def qr_r(self, A):
        A = np.ascontiguousarray(A, np.complex128)
        m, n = A.shape
        R = np.zeros((n, n), np.complex128)
        self._check(self.lib.ttfp_qr_r(self.ctx, m, n, _dp(A.view(np.float64)), _dp(R.view(np.float64))))
        return R

    def maxvol(self, A, delta=1e-2):
        A = np.ascontiguousarray(A, np.complex128)
        m, r = A.shape
        rows = np.zeros(r, np.int32)
        B = np.zeros((m, r), np.complex128)
        self._check(self.lib.ttfp_maxvol(self.ctx, m, r, _dp(A.view(np.float64)), float(delta), _ip(rows),
                                         _dp(B.view(np.float64))))
        return rows, B
