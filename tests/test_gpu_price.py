"""GPU TT-cross prices, through the C ABI, against the dense-grid oracle and closed forms."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import fourier as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pricer():
    import paper_2203_02804_amd as ttfp
    p = ttfp.Pricer(0)
    yield p
    p.close()


def oracle_grid(opt, N, L=None, alpha=None):
    """The oracle's per-term grid as explicit arrays for the GPU call."""
    _, grids = F.term_grids(opt, N, L, alpha)
    return np.array([g[0] for g in grids]), np.array([g[1] for g in grids])


def test_d1_black_scholes(pricer):
    for payoff in ("call_max", "put_max"):
        o = W.option(1, [100.0], 100.0, 1.0, 0.05, [0.2], [[1.0]], payoff)
        Ls, As = oracle_grid(o, 128)
        g = dict(W.grid(128, tol=1e-12, max_rank=4), L=Ls, alpha=As)
        p, ranks, info, rc = pricer.price(o, g)
        ref = F.dense_price(o, 128, Ls, As)
        assert abs(p / ref - 1) < 1e-13
        bs = CF.bs_call(100, 100, 1, 0.05, 0.2) if payoff == "call_max" else CF.bs_put(100, 100, 1, 0.05, 0.2)
        assert abs(p / bs - 1) < 1e-10
        assert ranks.tolist() == [[1, 1]]


def test_config1_literal_grid_parity(pricer):
    """Configuration 1 on its literal grid (N=64, L=40, |alpha|=2) at a rank that resolves it."""
    opt, g = W.config1()
    ref = F.dense_price(opt, 64, 40.0, 2.0)
    p, ranks, info, rc = pricer.price(opt, dict(g, max_rank=32))
    assert abs(p / ref - 1) < 1e-8, (p, ref, ranks, info)
    assert info["converged"]
    # on this symmetric grid the dense sum's imaginary part is ~1e-15 of its real part, so the
    # train's imaginary part is approximation error alone, bounded like the real part's (1e-8)
    # and in practice an order below it
    assert info["imag_rel"] < 1e-9


def test_config1_rank_cap_flagged(pricer):
    import paper_2203_02804_amd as ttfp
    opt, g = W.config1()       # max rank 8 binds on the second term
    ref = F.dense_price(opt, 64, 40.0, 2.0)
    p, ranks, info, rc = pricer.price(opt, g)
    assert rc == ttfp.TTFP_ENOTCONV and info["rank_capped"]
    assert np.max(ranks) <= 8
    assert abs(p / ref - 1) < 1e-3


def test_config1_closed_form(pricer):
    opt, _ = W.config1()
    stulz = CF.stulz_call_max(100, 100, 100, 1, 0.05, 0.2, 0.3, 0.5)
    g = W.grid(64, tol=1e-11, max_rank=48)          # automatic L / alpha
    p, ranks, info, rc = pricer.price(opt, g)
    assert abs(p / stulz - 1) < 1e-6, (p, stulz)
    ref = F.dense_price(opt, 64, tol=1e-11)
    assert abs(p / ref - 1) < 1e-8


@pytest.mark.parametrize("payoff", ["call_max", "put_max", "call_min"])
def test_d2_payoffs_against_dense(pricer, payoff):
    opt, _ = W.config1(payoff)
    opt = dict(opt, S0=[95.0, 104.0], sigma=[0.25, 0.18])
    Ls, As = oracle_grid(opt, 48)
    ref = F.dense_price(opt, 48, Ls, As)
    p, ranks, info, rc = pricer.price(opt, dict(W.grid(48, tol=1e-11, max_rank=48), L=Ls, alpha=As))
    assert abs(p / ref - 1) < 1e-8, (payoff, p, ref, ranks)


def test_d3_one_factor(pricer):
    for payoff in ("call_max", "put_max"):
        opt = W.option(3, [95.0, 100.0, 110.0], 100.0, 0.8, 0.03, [0.25, 0.2, 0.3],
                       W.equicorrelation(3, 1 / 3), payoff)
        N = 96
        ref = F.dense_price(opt, N, tol=1e-10)
        p, ranks, info, rc = pricer.price(opt, W.grid(N, tol=1e-10, max_rank=64))
        assert abs(p / ref - 1) < 1e-8, (payoff, p, ref, ranks, info)
        exact = CF.one_factor_price(opt["S0"], opt["K"], opt["T"], opt["r"], opt["sigma"], 1 / 3, payoff)
        assert abs(p / exact - 1) < 1e-7


def test_d4_random_correlation_ragged_grid(pricer):
    opt = W.random_small_options(1, seed=31, d_choices=(3,))[0]
    opt = W.option(4, opt["S0"] + [101.0], 100.0, opt["T"], opt["r"], opt["sigma"] + [0.27],
                   W.wishart_correlation(np.random.Generator(np.random.PCG64(5)), 4, 12), "call_max")
    N = 21                                          # odd, ragged against every tile size
    g = dict(W.grid(N, tol=1e-10, max_rank=64), L=10.0, alpha=1.5)
    ref = F.dense_price(opt, N, 10.0, 1.5)
    p, ranks, info, rc = pricer.price(opt, g)
    assert abs(p / ref - 1) < 1e-8, (p, ref, ranks, info)


def test_d5_small_grid(pricer):
    opt, _ = W.config2(corr_kind="beta")
    N = 16
    g = dict(W.grid(N, tol=1e-10, max_rank=64), L=8.0, alpha=1.5)
    ref = F.dense_price(opt, N, 8.0, 1.5)
    p, ranks, info, rc = pricer.price(opt, g)
    assert abs(p / ref - 1) < 1e-8, (p, ref, ranks, info)


def test_tt_interpolates_last_fibers_and_approximates_elsewhere(pricer):
    opt = W.random_small_options(1, seed=41, d_choices=(3,))[0]
    N = 32
    Ls, As = oracle_grid(opt, N)
    p, ranks, info, rc = pricer.price(opt, dict(W.grid(N, tol=1e-11, max_rank=48), L=Ls, alpha=As))
    ts, _ = F.term_grids(opt, N)
    rng = np.random.Generator(np.random.PCG64(3))
    for t, term in enumerate(ts):
        idx = rng.integers(0, N, size=(400, 3))
        tt = pricer.tt_values(t, idx)
        ref = F.integrand_at(term, N, Ls[t], As[t], idx)
        full = np.array(np.unravel_index(np.arange(N ** 3), (N,) * 3)).T
        fmax = np.max(np.abs(F.integrand_at(term, N, Ls[t], As[t], full)))
        assert np.max(np.abs(tt - ref)) < 1e-7 * fmax


def test_batch_matches_single(pricer):
    opts = W.random_small_options(6, seed=51, d_choices=(1, 2, 3))
    grid = dict(W.grid(32, tol=1e-11, max_rank=32), L=16.0, alpha=1.5)
    single = [pricer.price(o, grid)[0] for o in opts]
    batch, status = pricer.price_batch(opts, grid)
    assert np.allclose(batch, single, rtol=1e-9, atol=0)
    for o, p in zip(opts, batch):
        ref = F.dense_price(o, 32, 16.0, 1.5)
        assert abs(p / ref - 1) < 1e-8


def test_invalid_input_errors(pricer):
    import paper_2203_02804_amd as ttfp
    opt, g = W.config1()
    with pytest.raises(ttfp.TTFPError):
        pricer.price(dict(opt, sigma=[0.2, -0.1]), g)
    with pytest.raises(ttfp.TTFPError):
        pricer.price(opt, dict(g, max_rank=65))
    with pytest.raises(ttfp.TTFPError):
        pricer.price(opt, dict(g, N=2048))


def test_precision_flag_on_too_coarse_grid(pricer):
    import paper_2203_02804_amd as ttfp
    opt = W.option(3, [95.0, 100.0, 110.0], 100.0, 0.8, 0.03, [0.25, 0.2, 0.3], W.equicorrelation(3, 1 / 3))
    g = dict(W.grid(48, tol=1e-13, max_rank=48), L=30.0, alpha=6.0)     # a much too large shift
    p, ranks, info, rc = pricer.price(opt, g)
    det = F.dense_price(opt, 48, 30.0, 6.0, details=True)
    assert det["kappa"] > 500                      # the oracle's own cancellation factor
    assert det["kappa"] / 100 < info["kappa"] < det["kappa"] * 100   # the pricer's estimate
    assert rc != ttfp.TTFP_OK                       # kappa * eps exceeds tol


def test_tt_export_matches_tt_values_and_index_sets(pricer):
    opt = W.random_small_options(1, seed=61, d_choices=(3,))[0]
    N, R = 32, 24
    g = W.grid(N, tol=1e-10, max_rank=R)
    p, ranks, info, rc = pricer.price(opt, g)
    d = opt["d"]
    rng = np.random.Generator(np.random.PCG64(9))
    for t in range(ranks.shape[0]):
        ex = pricer.tt_export(t, d, R, N)
        assert ex["ranks"].tolist() == ranks[t].tolist()
        for k, G in enumerate(ex["cores"]):
            assert G.shape == (ranks[t][k], N, ranks[t][k + 1])
        idx = rng.integers(0, N, size=(64, d))
        vals = np.empty(len(idx), complex)
        for q, ix in enumerate(idx):
            v = np.ones(1, complex)
            for k, G in enumerate(ex["cores"]):
                v = v @ G[:, ix[k], :]
            vals[q] = v[0]
        ref = pricer.tt_values(t, idx)
        # the two contraction orders round differently; a wrong layout would differ at O(1)
        assert np.allclose(vals, ref, rtol=1e-8, atol=1e-11 * np.max(np.abs(ref)))
        # the final index sets: in range, distinct, and nested (I_{k+1} extends I_k, J_k extends J_{k+1})
        for k in range(1, d):
            I, J = ex["I"][k], ex["J"][k]
            assert I.shape[1] == k and J.shape[1] == d - k
            assert I.size == 0 or (I.min() >= 0 and I.max() < N)
            assert J.min() >= 0 and J.max() < N
            assert len(np.unique(J, axis=0)) == len(J)
            if k + 1 < d:
                prev = {tuple(row) for row in ex["J"][k + 1]}
                assert all(tuple(row[1:]) in prev for row in J)


# ---- the call on the minimum in the paper's own form: one term in asset coordinates with the
# joint single-strip transform (Sec. III.C min transform under Eq. main)

def test_min_strip_integrand_entries(pricer):
    opt = W.option(3, [95.0, 102.0, 108.0], 100.0, 0.8, 0.02, [0.25, 0.2, 0.3], W.sigma_beta(3, 0.5),
                   "call_min_strip")
    N = 50
    ts, grids = F.term_grids(opt, N, alpha=5.0 / 3)
    Ls, As = np.array([g[0] for g in grids]), np.array([g[1] for g in grids])
    rng = np.random.Generator(np.random.PCG64(8))
    idx = rng.integers(0, N, size=(500, 3))
    gpu = pricer.eval_integrand(opt, dict(W.grid(N), L=Ls, alpha=As), 0, idx)
    ref = F.integrand_at(ts[0], N, Ls[0], As[0], idx)
    assert np.max(np.abs(gpu - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,N", [(2, 64), (3, 48)])
def test_min_strip_against_dense(pricer, d, N):
    if d == 2:
        opt, _ = W.config1("call_min_strip")
    else:
        opt = W.option(3, [95.0, 102.0, 108.0], 100.0, 0.8, 0.02, [0.25, 0.2, 0.3], W.sigma_beta(3, 0.5),
                       "call_min_strip")
    Ls, As = oracle_grid(opt, N)
    g = dict(W.grid(N, tol=1e-11, max_rank=48, max_sweeps=6), L=Ls, alpha=As)
    p, ranks, info, rc = pricer.price(opt, g)
    ref = F.dense_price(opt, N, Ls, As)
    print(f"min strip d={d} N={N}: rel {p / ref - 1:+.2e} status {rc} ranks {ranks.tolist()}", flush=True)
    assert ranks.shape == (1, d + 1)
    assert abs(p / ref - 1) < 1e-8


def test_min_strip_one_factor_d5(pricer):
    opt = W.config2_batch(1, seed=77, corr_kind="beta")[0]
    opt = dict(opt, payoff="call_min_strip")
    ref = CF.one_factor_price(opt["S0"], opt["K"], opt["T"], opt["r"], opt["sigma"], 0.5 / 1.5, "call_min")
    p, ranks, info, rc = pricer.price(opt, W.grid(128, tol=1e-8, max_rank=48, max_sweeps=6))
    print(f"min strip d=5 N=128: rel {p / ref - 1:+.2e} status {rc} max rank {ranks.max()} err_est {info['err_est']:.1e}",
          flush=True)
    assert abs(p / ref - 1) < 1e-4
    if rc == 0:
        assert abs(p / ref - 1) < 1e-6
