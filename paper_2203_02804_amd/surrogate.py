"""Learned price surrogate on top of the tensor-train pricer.

An ensemble of MLPs (22 inputs -> 4 x 256 SiLU -> 1, BF16 weights and activations, FP32
accumulation, FP32 master weights, Adam) runs on the library's own HIP kernels
(ttfp_mlp_*). It learns the residual of the price over a closed-form control variate
(the largest single-asset Black-Scholes call), from prices the TT path generates.
At inference one fused kernel runs every model on a block of rows and forms, on the device,
the ensemble mean, its spread, and the gate: the spread scaled by a factor calibrated on
held-out TT prices estimates each row's error, and rows whose estimate exceeds the relative
gate are re-priced by the TT path (the fallback, which also judges the surrogate's error).
The host only prepares the input features and reads the gate's mask to pick the fallback rows.

Inputs for d assets: log(S0/K) (d), sigma (d), strictly lower Cholesky entries of the
correlation (d(d-1)/2), T, r -- 22 numbers for d = 5.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import TTFPError, load


def features(options):
    rows = []
    for o in options:
        d = o["d"]
        Lc = np.linalg.cholesky(np.asarray(o["corr"], float))
        low = [Lc[i, j] for i in range(d) for j in range(i)]
        rows.append(np.concatenate([np.log(np.asarray(o["S0"]) / o["K"]), np.asarray(o["sigma"]), low,
                                    [o["T"], o["r"]]]))
    return np.asarray(rows, np.float64)


class MLP:
    """Binding of the ttfp_mlp C ABI (an ensemble of identical-shape networks)."""

    def __init__(self, n_in, width=256, depth=4, n_models=4, max_batch=65536, seed=0, device=0, stream=None):
        import torch

        self.lib = load()
        lib = self.lib
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        lib.ttfp_mlp_create.argtypes = [P(vp), ctypes.c_int, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_uint64]
        lib.ttfp_mlp_destroy.argtypes = [vp]
        lib.ttfp_mlp_n_params.argtypes = [vp, P(ctypes.c_int64)]
        lib.ttfp_mlp_get_params.argtypes = [vp, ctypes.c_int, P(ctypes.c_float)]
        lib.ttfp_mlp_set_params.argtypes = [vp, ctypes.c_int, P(ctypes.c_float)]
        lib.ttfp_mlp_forward.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp]
        lib.ttfp_mlp_grad.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, P(ctypes.c_float), P(ctypes.c_float)]
        lib.ttfp_mlp_train_step.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_float, P(ctypes.c_float)]
        lib.ttfp_mlp_predict.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_float, ctypes.c_float, vp, vp, vp]
        lib.ttfp_mlp_control_variate.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp]
        lib.ttfp_mlp_last_error.argtypes = [vp]
        lib.ttfp_mlp_last_error.restype = ctypes.c_char_p
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.n_in, self.width, self.depth, self.n_models, self.max_batch = n_in, width, depth, n_models, max_batch
        self.h = ctypes.c_void_p()
        rc = lib.ttfp_mlp_create(ctypes.byref(self.h), device, ctypes.c_void_p(stream.cuda_stream), n_in, width, depth,
                                 n_models, max_batch, seed)
        if rc != 0:
            raise TTFPError(rc, "ttfp_mlp_create failed")
        n = ctypes.c_int64(0)
        lib.ttfp_mlp_n_params(self.h, ctypes.byref(n))
        self.n_params = n.value

    def close(self):
        if self.h:
            self.lib.ttfp_mlp_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise TTFPError(rc, self.lib.ttfp_mlp_last_error(self.h).decode())
        return rc

    def get_params(self, model):
        p = np.zeros(self.n_params, np.float32)
        self._check(self.lib.ttfp_mlp_get_params(self.h, model, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def set_params(self, model, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.n_params
        self._check(self.lib.ttfp_mlp_set_params(self.h, model, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    @staticmethod
    def _dev(x):
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        return ctypes.c_void_p(x.data_ptr())

    def forward(self, model, x):
        import torch
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        self._check(self.lib.ttfp_mlp_forward(self.h, model, x.shape[0], self._dev(x), self._dev(y)))
        return y

    def predict(self, x, cv, scale, factor, gate):
        """Fused ensemble inference with the gate on the device: device tensors (mean, spread, ok)
        of price_m = cv + scale * y_m over the models (see ttfp_mlp_predict)."""
        import torch
        B = x.shape[0]
        mean = torch.empty(B, dtype=torch.float32, device=x.device)
        spread = torch.empty_like(mean)
        ok = torch.empty(B, dtype=torch.int32, device=x.device)
        self._check(self.lib.ttfp_mlp_predict(self.h, B, self._dev(x), self._dev(cv), self._dev(scale), float(factor),
                                              float(gate), self._dev(mean), self._dev(spread), ctypes.c_void_p(ok.data_ptr())))
        return mean, spread, ok

    def control_variate(self, S0, sigma, K, T, r):
        """max_j of the single-asset Black-Scholes calls on the device (device FP32 tensors)."""
        import torch
        B, d = S0.shape
        cv = torch.empty(B, dtype=torch.float32, device=S0.device)
        self._check(self.lib.ttfp_mlp_control_variate(self.h, B, d, self._dev(S0), self._dev(sigma), self._dev(K),
                                                      self._dev(T), self._dev(r), self._dev(cv)))
        return cv

    def grad(self, model, x, t):
        g = np.zeros(self.n_params, np.float32)
        loss = ctypes.c_float(0.0)
        self._check(self.lib.ttfp_mlp_grad(self.h, model, x.shape[0], self._dev(x), self._dev(t),
                                           g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, model, x, t, lr):
        loss = ctypes.c_float(0.0)
        self._check(self.lib.ttfp_mlp_train_step(self.h, model, x.shape[0], self._dev(x), self._dev(t), float(lr),
                                                 ctypes.byref(loss)))
        return loss.value


class Surrogate:
    """Ensemble surrogate of the TT price with an error gate and TT fallback."""

    def __init__(self, d=5, width=256, depth=4, n_models=4, max_batch=65536, seed=0, device=0):
        self.d = d
        self.n_in = 2 * d + d * (d - 1) // 2 + 2
        self.net = MLP(self.n_in, width, depth, n_models, max_batch, seed, device)
        self.n_models = n_models
        self.mu = None
        self.sd = None
        self.tscale = 1.0
        self.factor = 3.0
        self.device = device

    # -- data transforms
    def _x(self, options):
        import torch
        f = features(options)
        if self.mu is None:
            self.mu = f.mean(axis=0)
            self.sd = f.std(axis=0) + 1e-12
        return torch.tensor((f - self.mu) / self.sd, dtype=torch.float32, device=f"cuda:{self.device}").contiguous()

    def _device_inputs(self, options):
        """Normalised features, control variate and price scale of each row, on the device."""
        import torch
        dev = f"cuda:{self.device}"
        X = self._x(options)
        f32 = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=torch.float32, device=dev).contiguous()
        S0 = f32([o["S0"] for o in options])
        sig = f32([o["sigma"] for o in options])
        K = f32([o["K"] for o in options])
        cv = self.net.control_variate(S0, sig, K, f32([o["T"] for o in options]), f32([o["r"] for o in options]))
        return X, cv, (K * self.tscale).contiguous()

    def _target(self, options, prices):
        import torch
        dev = f"cuda:{self.device}"
        f32 = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=torch.float32, device=dev).contiguous()
        cv = self.net.control_variate(f32([o["S0"] for o in options]), f32([o["sigma"] for o in options]),
                                      f32([o["K"] for o in options]), f32([o["T"] for o in options]),
                                      f32([o["r"] for o in options])).double().cpu().numpy()
        K = np.array([o["K"] for o in options])
        return (np.asarray(prices) - cv) / K

    def fit(self, options, prices, steps=2000, batch=1024, lr=1e-3, holdout=0.1, seed=0, log_every=0):
        """Trains every ensemble member on the TT prices (each with its own shuffle), then
        calibrates the spread factor on the held-out part."""
        import torch
        n = len(options)
        rng = np.random.Generator(np.random.PCG64(seed))
        perm = rng.permutation(n)
        n_hold = max(1, int(holdout * n))
        hold, train = perm[:n_hold], perm[n_hold:]
        opts_tr = [options[i] for i in train]
        self.mu = None
        X = self._x(opts_tr)
        y = self._target(opts_tr, np.asarray(prices)[train])
        self.tscale = float(np.std(y)) + 1e-12
        T = torch.tensor(y / self.tscale, dtype=torch.float32, device=X.device)
        hist = []
        B = min(batch, X.shape[0])
        for m in range(self.n_models):
            g = torch.Generator(device="cpu").manual_seed(seed * 1000 + m)
            for s in range(steps):
                idx = torch.randint(0, X.shape[0], (B,), generator=g).to(X.device)
                xb = X.index_select(0, idx).contiguous()
                tb = T.index_select(0, idx).contiguous()
                frac = s / max(steps - 1, 1)
                lr_s = lr * 0.5 * (1 + math.cos(math.pi * frac))       # cosine schedule
                loss = self.net.train_step(m, xb, tb, max(lr_s, lr * 1e-3))
                if log_every and s % log_every == 0:
                    hist.append((m, s, loss))
        # calibration on held-out TT prices
        opts_h = [options[i] for i in hold]
        mean, spread = self.predict(opts_h)
        err = np.abs(mean - np.asarray(prices)[hold])
        ratio = err / np.maximum(spread, 1e-300)
        self.factor = float(np.quantile(ratio, 0.99)) if len(ratio) > 1 else 3.0
        return dict(history=hist, holdout_rel_err=err / np.abs(np.asarray(prices)[hold]), factor=self.factor)

    def predict(self, options):
        """Ensemble mean price and ensemble spread (standard deviation), both in price units,
        from the fused ensemble kernel (host arrays)."""
        X, cv, scale = self._device_inputs(options)
        mean, spread, _ = self.net.predict(X, cv, scale, self.factor, 0.0)
        return mean.double().cpu().numpy(), spread.double().cpu().numpy()

    def price(self, options, pricer, grid, rel_gate=1e-4):
        """Surrogate prices where factor * spread <= rel_gate * |price| (decided on the device),
        TT prices elsewhere. Returns (prices, served_by_surrogate mask, status): status holds the
        TT return code of every fallback row and 0 for the rows the surrogate served."""
        X, cv, scale = self._device_inputs(options)
        mean, spread, okd = self.net.predict(X, cv, scale, self.factor, rel_gate)
        ok = okd.cpu().numpy().astype(bool)
        out = mean.double().cpu().numpy()
        status = np.zeros(len(options), np.int32)
        fb = np.nonzero(~ok)[0]
        if len(fb):
            p, st = pricer.price_batch([options[i] for i in fb], grid)
            out[fb] = p
            status[fb] = st
        return out, ok, status
