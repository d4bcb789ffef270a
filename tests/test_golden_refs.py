"""The stored one-factor references of the benchmark workload against the oracle that wrote them.

tests/golden/one_factor_config2prime.json holds, per seed, the one-factor semi-closed-form
prices (Sec. V.B correlation family Sigma(0.5)) of config2_batch(192, seed, 'beta'); the
benchmark reads prefixes of these lists for smaller batches.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "one_factor_config2prime.json")


@pytest.fixture(scope="module")
def stored():
    with open(GOLDEN) as f:
        return json.load(f)


def test_layout(stored):
    assert stored["batch"] == 192
    assert len(stored["batches"]) == 32
    assert all(len(v) == 192 for v in stored["batches"].values())
    assert abs(stored["rho"] - 0.5 / 1.5) < 1e-15


@pytest.mark.parametrize("seed", [2203, 7203])
def test_sampled_entries_match_the_oracle(stored, seed):
    opts = W.config2_batch(192, seed=seed, corr_kind="beta")
    for i in (0, 127, 128, 191):            # both sides of the former 128-option file
        o = opts[i]
        ref = CF.one_factor_price(o["S0"], o["K"], o["T"], o["r"], o["sigma"], stored["rho"], "call_max")
        assert ref == pytest.approx(stored["batches"][str(seed)][i], rel=1e-12)


def test_smaller_batches_are_prefixes():
    # the benchmark's --batch n takes the first n references of a seed
    a = W.config2_batch(64, seed=3203, corr_kind="beta")
    b = W.config2_batch(192, seed=3203, corr_kind="beta")
    for x, y in zip(a, b[:64]):
        assert np.array_equal(np.asarray(x["S0"]), np.asarray(y["S0"]))
        assert np.array_equal(np.asarray(x["sigma"]), np.asarray(y["sigma"]))
        assert x["T"] == y["T"] and x["K"] == y["K"]
