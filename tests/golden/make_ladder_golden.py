"""Writes tests/golden/ladder.json: exact prices of a market ladder around the first option of the
d = 5 one-factor batch (correlation Sigma(0.5), Sec. V.B, Eq. covmat; seed 0 of the stored one-factor
batches): 1024 points (spots scaled per asset by U[0.85, 1.15], strikes U[85, 115], rates
U[0, 0.06], seed 7), each priced by the one-factor semi-closed form (~1e-12).

Calls only the oracle. Run:  python tests/golden/make_ladder_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import closed_forms as CF  # noqa: E402

N_POINTS = 1024


def main():
    with open(os.path.join(HERE, "one_factor_config2prime.json")) as f:
        seed = sorted(int(s) for s in json.load(f)["batches"])[0]
    base = W.config2_batch(1, seed=seed, corr_kind="beta")[0]
    S0, K, r = W.ladder_points(base, N_POINTS, seed=7)
    t0 = time.time()
    prices = [CF.one_factor_price(S0[p], K[p], base["T"], r[p], base["sigma"], 0.5 / 1.5, base["payoff"])
              for p in range(N_POINTS)]
    out = {"description": "one-factor prices of a 1024-point ladder around the first option of the d=5 "
                          "Sigma(0.5) batch", "batch_seed": seed, "ladder_seed": 7, "prices": prices,
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, "ladder.json"), "w") as f:
        json.dump(out, f)
    print(out["seconds"], prices[:3])


if __name__ == "__main__":
    main()
