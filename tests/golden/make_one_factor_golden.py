"""Writes tests/golden/one_factor_config2prime.json: exact prices of the d=5 call-on-max
options of the one-factor companion workload (the paper's correlation family Sigma(beta=0.5),
Sec. V.B, Eq. covmat, with the d=5 configuration's other distributions), for the seeds the
benchmark and the full-size GPU test draw.

The reference is the one-factor semi-closed form in oracle/closed_forms.py (conditioning on
the common factor reduces the d-dimensional expectation to a 2-D quadrature, accurate to
~1e-12). Calls only the oracle. Run:  python tests/golden/make_one_factor_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import closed_forms as CF  # noqa: E402

BATCH = 192
SEEDS = [2203 + 1000 * s for s in range(32)]    # benchmark batches (warm-up + timed steps)


def main():
    rho = 0.5 / 1.5                            # off-diagonal of Sigma(0.5)
    out = {"description": "one-factor semi-closed-form prices of config2_batch(n, seed, corr_kind='beta') "
                          "options (d=5 call on max, Sigma(0.5) correlation)",
           "rho": rho, "batch": BATCH, "batches": {}}
    t0 = time.time()
    for seed in SEEDS:
        opts = W.config2_batch(BATCH, seed=seed, corr_kind="beta")
        out["batches"][str(seed)] = [CF.one_factor_price(o["S0"], o["K"], o["T"], o["r"], o["sigma"], rho, "call_max")
                                     for o in opts]
        print(seed, f"{time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "one_factor_config2prime.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
