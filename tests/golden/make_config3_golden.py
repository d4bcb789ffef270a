"""Writes tests/golden/config3.json: oracle references for the d=20 call-on-max configuration
(N=256 per dimension, tol 1e-8, max rank 64).

  corr=beta     the one-factor companion (the paper's correlation family Sigma(0.5), Sec. V.B,
                Eq. covmat, off-diagonal 1/3): the one-factor semi-closed form, ~1e-12
  corr=wishart  the literal configuration (seeded Wishart correlation): no dense grid (256^20
                points) and no closed form, so Monte Carlo with 10^8 exact-terminal paths
                (antithetic pairs) and its standard error

Calls only the oracle. Run:  python tests/golden/make_config3_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import closed_forms as CF  # noqa: E402
from oracle import mc as MC  # noqa: E402

MC_PATHS = 10 ** 8


def main():
    out = {"description": "references for config3 (d=20 call on max): one-factor price of the Sigma(0.5) "
                          "companion, 1e8-path Monte Carlo of the Wishart configuration",
           "cases": []}
    t0 = time.time()
    o, _ = W.config3(corr_kind="beta")
    p = CF.one_factor_price(o["S0"], o["K"], o["T"], o["r"], o["sigma"], 0.5 / 1.5, "call_max")
    out["cases"].append({"workload": "config3 seed 2804 corr=beta", "method": "one-factor", "price": p,
                         "seconds": time.time() - t0})
    print("beta", p, flush=True)
    t0 = time.time()
    o, _ = W.config3(corr_kind="wishart")
    p, se = MC.mc_price(o, MC_PATHS, seed=2804)
    out["cases"].append({"workload": "config3 seed 2804 corr=wishart", "method": f"monte carlo {MC_PATHS} paths",
                         "price": p, "stderr": se, "seconds": time.time() - t0})
    print("wishart", p, se, flush=True)
    with open(os.path.join(HERE, "config3.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
