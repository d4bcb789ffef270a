"""Writes tests/golden/book_slice.json: oracle references for a slice of the batched book
(configuration 4: call on the max of d ~ U{2..10} assets, N ~ U{64, 128, 256} per dimension,
seed 22030), priced with Greeks in one batched launch by the GPU test.

  d <= 3 and (d = 4, N = 64): the book's own Wishart correlation; the dense-grid Fourier price
      on the automatic grid of tol 1e-8 (the grid is stored) and central finite-difference
      Greeks of that fixed-grid price (relative S0 bump 1e-4, absolute sigma bump 1e-4)
  d >= 5: the same draws with the correlation replaced by the paper's Sigma(0.5) (Sec. V.B,
      Eq. covmat, off-diagonal 1/3), where the one-factor semi-closed form is exact; Greeks by
      central differences of that form (same bumps)

Calls only the oracle. Run:  python tests/golden/make_book_golden.py
"""
import copy
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import closed_forms as CF  # noqa: E402
from oracle import fourier as F  # noqa: E402
from oracle import greeks as G  # noqa: E402

TOL = 1e-8
H = 1e-4
RHO = 0.5 / 1.5


def one_factor(o):
    return CF.one_factor_price(o["S0"], o["K"], o["T"], o["r"], o["sigma"], RHO, "call_max")


def one_factor_greeks(o):
    d = o["d"]
    delta, vega = np.zeros(d), np.zeros(d)
    for j in range(d):
        up, dn = copy.deepcopy(o), copy.deepcopy(o)
        up["S0"][j] *= 1 + H
        dn["S0"][j] *= 1 - H
        delta[j] = (one_factor(up) - one_factor(dn)) / (2 * H * o["S0"][j])
        up, dn = copy.deepcopy(o), copy.deepcopy(o)
        up["sigma"][j] += H
        dn["sigma"][j] -= H
        vega[j] = (one_factor(up) - one_factor(dn)) / (2 * H)
    return delta, vega


def main():
    opts, Ns = W.config4()
    picks = {"dense": [], "d4": [], "beta": []}
    for i, (o, N) in enumerate(zip(opts, Ns)):
        d = o["d"]
        if d <= 3 and len(picks["dense"]) < 16:
            picks["dense"].append(i)
        elif d == 4 and N == 64 and len(picks["d4"]) < 4:
            picks["d4"].append(i)
        elif d >= 5 and len(picks["beta"]) < 16:
            picks["beta"].append(i)
    out = {"description": "slice of config4 (seed 22030) with oracle prices and finite-difference Greeks",
           "tol": TOL, "bump": H, "cases": []}
    t0 = time.time()
    for i in picks["dense"] + picks["d4"]:
        o, N = copy.deepcopy(opts[i]), Ns[i]
        Ls, As = G.fixed_grid(o, N, tol=TOL)
        p = F.dense_price(o, N, Ls, As)
        dl, vg = G.fd_greeks(o, N, Ls, As, h=H)
        out["cases"].append({"index": i, "d": o["d"], "N": N, "corr": "wishart", "method": "dense",
                             "L": Ls.tolist(), "alpha": As.tolist(), "price": p, "delta": dl.tolist(),
                             "vega": vg.tolist()})
        print(i, o["d"], N, p, f"{time.time() - t0:.0f} s", flush=True)
    for i in picks["beta"]:
        o, N = copy.deepcopy(opts[i]), Ns[i]
        o["corr"] = W.sigma_beta(o["d"], 0.5)
        p = one_factor(o)
        dl, vg = one_factor_greeks(o)
        out["cases"].append({"index": i, "d": o["d"], "N": N, "corr": "beta", "method": "one-factor",
                             "price": p, "delta": dl.tolist(), "vega": vg.tolist()})
        print(i, o["d"], N, p, f"{time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "book_slice.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
