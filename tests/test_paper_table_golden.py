"""Pins for the stored references of the paper's call-on-min experiment
(tests/golden/paper_table.json): the one-factor prices and the dense grid sums agree where the
grid's discretisation error is small, and the stored values are what the oracle computes."""
import json
import os

import workloads as W
from oracle import closed_forms as CF
from oracle import fourier as F

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_table.json")


def test_stored_references_are_the_oracles():
    with open(GOLDEN) as f:
        gold = json.load(f)
    c = next(c for c in gold["table"] if c["d"] == 2)
    o, g = W.paper_experiment(2)
    assert abs(F.dense_price(o, g["N"], g["L"], g["alpha"]) / c["dense"] - 1) < 1e-13
    assert abs(CF.one_factor_price(o["S0"], o["K"], o["T"], o["r"], o["sigma"], 0.5 / 1.5, "call_min")
               / c["one_factor"] - 1) < 1e-12


def test_grid_sum_approaches_the_exact_price():
    # the experiment's grid (N = 50, Table I spacing) against the exact price: 1e-9 at d = 2 and
    # 1e-5 at d = 3 for every correlation of the bond-dimension study, 1e-3 at d = 4
    with open(GOLDEN) as f:
        gold = json.load(f)
    bound = {2: 1e-9, 3: 1e-5, 4: 1e-3}
    for c in gold["table"] + gold["bond"]:
        if "dense" in c:
            assert abs(c["dense"] / c["one_factor"] - 1) < bound[c["d"]], c
