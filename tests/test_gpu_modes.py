"""Launch modes of the pricer: repeatability, hipGraph replay, launch tunings, autotuner."""
import numpy as np
import pytest

import workloads as W
from oracle import fourier as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pricer():
    import torch

    import paper_2203_02804_amd as ttfp
    s = torch.cuda.Stream()          # graph capture needs a stream other than the null stream
    p = ttfp.Pricer(0, stream=s)
    yield p
    p.close()


def _batch():
    opts = W.random_small_options(6, seed=404, d_choices=(2, 3))
    return opts, dict(W.grid(48, tol=1e-11, max_rank=48, max_sweeps=6), L=14.0, alpha=1.25)


def test_repeatable(pricer):
    opts, g = _batch()
    a, _ = pricer.price_batch(opts, g)
    b, _ = pricer.price_batch(opts, g)
    assert np.array_equal(a, b)


def test_result_independent_of_batch_composition(pricer):
    # d = 5 options whose crosses do not converge: every pivot decision must still be the
    # same whichever options share the launch
    opts = W.config5_options(24, seed=5, corr_kind="beta")
    g = W.grid(128, tol=1e-8, max_rank=48, max_sweeps=4)
    full, _ = pricer.price_batch(opts, g)
    again, _ = pricer.price_batch(opts, g)
    part, _ = pricer.price_batch(opts[5:15], g)
    assert np.array_equal(full, again)
    assert np.array_equal(full[5:15], part)


def test_graph_replay_matches_eager(pricer):
    opts, g = _batch()
    pricer.set_tuning(graph=0)
    eager, _ = pricer.price_batch(opts, g)
    pricer.set_tuning(graph=1)
    for _ in range(3):               # each call captures once and replays every half sweep
        graph, _ = pricer.price_batch(opts, g)
        assert np.array_equal(graph, eager)
    pricer.set_tuning(graph=0)


@pytest.mark.parametrize("rounds,lds,warm", [(0, 48, 1), (2, 76, 0), (3, 152, 1), (3, 152, 0), (5, 100, 1)])
def test_tunings_agree_with_the_oracle(pricer, rounds, lds, warm):
    opts, g = _batch()
    pricer.set_tuning(maxvol_rounds=rounds, tsqr_lds_kb=lds, maxvol_warm=warm)
    p, status = pricer.price_batch(opts, g)
    pricer.set_tuning(maxvol_rounds=3, tsqr_lds_kb=152, maxvol_warm=1)
    for o, v in zip(opts, p):
        ref = F.dense_price(o, 48, 14.0, 1.25)
        assert abs(v / ref - 1) < 1e-8


def test_autotuner_picks_a_valid_setting(pricer, tmp_path):
    from paper_2203_02804_amd import tuning
    opts, g = _batch()
    best, timings = tuning.tune(pricer, opts, g, reps=1, path=str(tmp_path / "t.json"))
    assert set(best) == set(tuning.CANDIDATES)
    assert len(timings) == 16
    entry = tuning.apply(pricer, opts[0]["d"], g["N"], g["max_rank"], path=str(tmp_path / "t.json"))
    assert entry is not None and pricer.get_tuning()["mm_waves"] == best["mm_waves"]
    pricer.set_tuning(graph=1, mm_waves=8, mm_panels=1, gram_threads=512)


def test_tile_shapes_agree_bit_for_bit(pricer):
    # the basis and interpolation products with 8 or 16 row panels per workgroup and the Gram
    # products with one or two tiles per wave: the same prices bit for bit
    opts, g = _batch()
    pricer.autotune = False
    pricer.set_tuning(mm_waves=8, gram_threads=512)
    p0, s0 = pricer.price_batch(opts, g)
    for mw, mp, gt in ((16, 1, 512), (8, 2, 512), (16, 2, 1024), (8, 1, 1024)):
        pricer.set_tuning(mm_waves=mw, mm_panels=mp, gram_threads=gt)
        p1, s1 = pricer.price_batch(opts, g)
        assert np.array_equal(p0, p1) and np.array_equal(s0, s1), (mw, mp, gt)
    pricer.set_tuning(mm_waves=8, mm_panels=1, gram_threads=512)
    pricer.autotune = True


def test_row_bound_of_the_checking_passes_is_exact(pricer):
    # skipping the rows that |B_ij|^2 <= |y_i|^2 max_j |A^-1 e_j|^2 clears changes nothing: the
    # same prices and statuses bit for bit, also on the headline workload's shape
    pricer.autotune = False
    for opts, g in (_batch(), (W.config2_batch(6, seed=2203, corr_kind="beta"),
                               W.grid(256, tol=1e-8, max_rank=64, max_sweeps=4))):
        pricer.set_tuning(interp_bound=0)
        p0, s0 = pricer.price_batch(opts, g)
        pricer.set_tuning(interp_bound=1)
        p1, s1 = pricer.price_batch(opts, g)
        assert np.array_equal(p0, p1) and np.array_equal(s0, s1)
    pricer.autotune = True
