"""Writes tests/golden/paper_table.json: oracle references for the paper's multi-asset experiment
(Sec. V.B: the call on the minimum, r = 0.3, sigma = 0.5, T = 1, S0 = K = 100, correlation
Sigma(beta), N = 50 nodes with the Table I spacing, shift 5 / d, single-strip transform in asset
coordinates).

  table     d = 2..10, 15 at beta = 0.5: the one-factor semi-closed form (the exact price, which
            the paper lacked beyond d = 4) and, for d <= 4, the dense grid sum at the experiment's
            grid (the quantity a converged cross reproduces)
  bond      d = 3, beta = 0.2, 0.5, 1 (the bond-dimension study): dense grid sum and one-factor price

Calls only the oracle. Run:  python tests/golden/make_paper_table_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import closed_forms as CF  # noqa: E402
from oracle import fourier as F  # noqa: E402


def case(d, beta, dense):
    o, g = W.paper_experiment(d, beta)
    rho = beta / (1.0 + beta)
    t0 = time.time()
    c = {"d": d, "beta": beta, "N": g["N"], "L": g["L"], "alpha": g["alpha"],
         "one_factor": CF.one_factor_price(o["S0"], o["K"], o["T"], o["r"], o["sigma"], rho, "call_min")}
    if dense:
        c["dense"] = F.dense_price(o, g["N"], g["L"], g["alpha"])
    c["seconds"] = time.time() - t0
    print(json.dumps(c), flush=True)
    return c


def main():
    out = {"description": "references for the paper's call-on-min experiment (Sec. V.B, Table I): one-factor "
                          "prices, and dense grid sums at the experiment's grid for d <= 4",
           "table": [case(d, 0.5, d <= 4) for d in W.PAPER_TABLE_DIMS],
           "bond": [case(3, b, True) for b in (0.2, 0.5, 1.0)]}
    with open(os.path.join(HERE, "paper_table.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
