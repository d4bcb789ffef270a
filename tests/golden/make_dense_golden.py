"""Writes tests/golden/dense_config2.json: the dense-grid oracle price of the d=5
call-on-max configurations on their full N=128 grids (5 terms x 128^5 points each).

Calls only the oracle (oracle/fourier.py, oracle/closed_forms.py); takes tens of minutes
on a multi-core host. Run:  python tests/golden/make_dense_golden.py
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


def main():
    out = {"description": "dense-grid Fourier price (oracle) on the automatic grid of the given tol, "
                          "N=128 per dimension, all 5 terms",
           "cases": []}
    for kind in ("wishart", "beta"):
        opt, g = W.config2(corr_kind=kind)
        t0 = time.time()
        det = F.dense_price(opt, g["N"], details=True, tol=g["tol"])
        case = {"workload": f"config2 seed 2203 corr={kind}", "N": g["N"], "tol": g["tol"],
                "price": det["price"], "imag": det["imag"], "abs_sum": det["abs_sum"],
                "seconds": time.time() - t0}
        if kind == "beta":
            case["one_factor"] = CF.one_factor_price(opt["S0"], opt["K"], opt["T"], opt["r"], opt["sigma"],
                                                     1 / 3, "call_max")
        out["cases"].append(case)
        print(json.dumps(case), flush=True)
    with open(os.path.join(HERE, "dense_config2.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
