"""The two-train variant (Sec. IV, Eq. braket; ttfp_price_two_trains): one cross of the
characteristic function and one of the payoff transform, priced by their exact inner product,
against the oracle's dense grid sums (the variant's exact-arithmetic value)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import fourier as F

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_table.json")


@pytest.fixture(scope="module")
def pricer():
    import paper_2203_02804_amd as ttfp
    p = ttfp.Pricer(0)
    yield p
    p.close()


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_paper_experiment_two_trains(pricer, gold, d):
    # the paper's own set-up: the call on the minimum in asset coordinates, D_phi and D_v caps
    opt, g = W.paper_experiment(d, max_rank=40)
    c = next(c for c in gold["table"] if c["d"] == d)
    p, rcf, rpay, info, rc = pricer.price_two_trains(opt, g, payoff_rank=40)
    rel = p / c["dense"] - 1
    print(f"two trains d={d}: rel {rel:+.2e} status {rc} D_phi {rcf.max()} D_v {rpay.max()} evals {info['n_evals']} "
          f"err_est {info['err_est']:.1e}", flush=True)
    assert abs(rel) <= 1e-8


def test_rotated_call_on_max_payoff_train_is_rank_one(pricer):
    # in the rotated coordinates of a call-on-max term the payoff transform is a product of
    # one-dimensional factors: its train has rank one
    opt, _ = W.config1()
    N = 64
    grids = np.array(F.term_grids(opt, N, tol=1e-10)[1])
    g = dict(W.grid(N, tol=1e-10, max_rank=32), L=grids[:, 0], alpha=grids[:, 1])
    p, rcf, rpay, info, rc = pricer.price_two_trains(opt, g, payoff_rank=8)
    ref = F.dense_price(opt, N, grids[:, 0], grids[:, 1])
    print(f"two trains config1: rel {p / ref - 1:+.2e} status {rc} payoff ranks {rpay.tolist()}", flush=True)
    assert abs(p / ref - 1) <= 1e-9
    assert rpay.max() == 1


def test_bond_dimension_of_the_characteristic_function(pricer, gold):
    # the paper's bond-dimension study (d = 3, D_v = 30): the error against the grid sum falls
    # with the characteristic function's rank cap D_phi, faster for weaker correlation
    for beta in (0.2, 0.5, 1.0):
        c = next(c for c in gold["bond"] if abs(c["beta"] - beta) < 1e-12)
        errs = {}
        for Dphi in (2, 4, 8, 16):
            e = []
            for seed in range(4):
                opt, g = W.paper_experiment(3, beta, max_rank=Dphi, seed=seed)
                p, _, _, _, _ = pricer.price_two_trains(opt, g, payoff_rank=30)
                e.append(abs(p / c["dense"] - 1))
            errs[Dphi] = float(np.mean(e))
        print(f"two trains beta={beta}: " + " ".join(f"D_phi={k}: {v:.1e}" for k, v in errs.items()), flush=True)
        assert errs[16] < 1e-6
        assert errs[2] > 100 * errs[16]


def test_two_trains_with_jumps(pricer):
    # with Merton jumps the jump factor belongs to the characteristic-function train only: the
    # payoff train of a rotated call-on-max term stays rank one and the price matches the grid sum.
    # Without the payoff's decay the characteristic function alone needs rank up to N here, so N
    # stays below the rank cap.
    opt = W.merton_options(1, seed=34, d_choices=(2,), payoffs=("call_max",))[0]
    N = 48
    grids = np.array(F.term_grids(opt, N, tol=1e-11)[1])
    g = dict(W.grid(N, tol=1e-11, max_rank=64, max_sweeps=16), L=grids[:, 0], alpha=grids[:, 1])
    p, rcf, rpay, info, rc = pricer.price_two_trains(opt, g, payoff_rank=8)
    ref = F.dense_price(opt, N, grids[:, 0], grids[:, 1])
    print(f"two trains merton: rel {p / ref - 1:+.2e} status {rc} D_phi {rcf.max()} payoff ranks {rpay.tolist()}",
          flush=True)
    assert rc == 0
    assert abs(p / ref - 1) <= 1e-8
    assert rpay.max() == 1
