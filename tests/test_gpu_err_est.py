"""The sampled error estimate of the cross (Sec. IV.B: relative 1-norm error of the tensor
train against the integrand on random grid points), computed on the GPU, against the same
measure recomputed on the CPU: the oracle's integrand at the same points (rebuilt from the
generator's published definition in oracle/rng.py) and the exported tensor trains evaluated
with NumPy."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fourier as F
from oracle import rng as RNG

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pricer():
    import paper_2203_02804_amd as ttfp
    p = ttfp.Pricer(0)
    yield p
    p.close()


def tt_eval(cores, idx):
    out = np.empty(idx.shape[0], complex)
    for p in range(idx.shape[0]):
        v = np.ones(1, complex)
        for k, G in enumerate(cores):
            v = v @ G[:, idx[p, k], :]
        out[p] = v[0]
    return out


CASES = [
    (W.config1()[0], 64, 16, 1e-10),
    (W.random_small_options(1, seed=17, d_choices=(3,))[0], 40, 12, 1e-8),
    (W.config2_batch(1, seed=2203, corr_kind="beta")[0], 32, 10, 1e-6),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_err_est_matches_cpu_recomputation(pricer, case):
    opt, N, R, tol = CASES[case]
    d = opt["d"]
    terms, grids = F.term_grids(opt, N, tol=tol)
    Ls = np.array([g[0] for g in grids])
    As = np.array([g[1] for g in grids])
    n_samp, seed = 3001, 5
    g = dict(W.grid(N, tol=tol, max_rank=R, max_sweeps=4, seed=seed), L=Ls, alpha=As, n_err_samples=n_samp)
    print(f"err_est case {case}: d={d} N={N} R={R}", flush=True)
    price, ranks, info, rc = pricer.price(opt, g)
    per = math.ceil(n_samp / len(terms))
    assert info["err_samples"] == per * len(terms)
    ea = ef = 0.0
    for t, term in enumerate(terms):
        ex = pricer.tt_export(t, d, R, N)
        pts = RNG.sample_points(seed, t, per, d, N)
        tt = tt_eval(ex["cores"], pts)
        f = F.integrand_at(term, N, Ls[t], As[t], pts)
        sc = F.term_scale(opt, Ls[t], N)
        ea += sc * np.sum(np.abs(tt - f))
        ef += sc * np.sum(np.abs(f))
    ref = ea / ef
    print(f"  err_est gpu {info['err_est']:.6e} cpu {ref:.6e} (status {rc})", flush=True)
    assert abs(info["err_est"] - ref) <= 1e-6 * ref + 1e-13


def test_err_est_off_and_batch_diag(pricer):
    opt, _ = W.config1()
    g = dict(W.grid(64, tol=1e-10, max_rank=16), n_err_samples=-1)
    _, _, info, _ = pricer.price(opt, g)
    assert math.isnan(info["err_est"]) and info["err_samples"] == 0
    # the batch reports, per option, the estimate a single-option call on the same option gives
    # (same kernels, same sample points, same tensor trains)
    opts = W.random_small_options(3, seed=23, d_choices=(2, 3))
    g2 = dict(W.grid(48, tol=1e-9, max_rank=12), n_err_samples=2000)
    prices, status = pricer.price_batch(opts, g2)
    for i, o in enumerate(opts):
        dg = pricer.batch_diag(i)
        nt = o["d"] if o["d"] > 1 else 1
        assert dg["err_samples"] == math.ceil(2000 / nt) * nt
        p1, _, info1, _ = pricer.price(o, g2)
        assert p1 == prices[i]
        assert 0.0 <= dg["err_est"] < 1.0
        assert abs(dg["err_est"] - info1["err_est"]) <= 1e-12 * info1["err_est"]


def test_certified_status(pricer):
    # certify = 1 keeps TTFP_OK only where the sampled bound err_est * kappa meets tol; every
    # other code is unchanged, and a certified price is within tol of the dense-grid oracle. At
    # N = 16 and a rank cap above N the trains can be exact (d <= 3), so the bound can be met;
    # at N = 64 with rank 8 it is not, and converged options are demoted.
    import paper_2203_02804_amd as ttfp
    opts = ([W.config1()[0]] + W.random_small_options(2, seed=3, d_choices=(1,))
            + W.random_small_options(3, seed=31, d_choices=(2, 3)))
    n_cert = 0
    for N, R in ((16, 20), (64, 8)):
        g = dict(W.grid(N, tol=1e-6, max_rank=R), n_err_samples=4000)
        # the oracle's grid, handed to both sides
        grids = [np.array(v) for v in (F.term_grids(o, N, tol=g["tol"])[1] for o in opts)]
        gl = [dict(g, L=G[:, 0], alpha=G[:, 1]) for G in grids]
        p0, s0 = pricer.price_batch(opts, gl)
        p1, s1 = pricer.price_batch(opts, [dict(x, certify=1) for x in gl])
        assert np.array_equal(p0, p1)
        for i, o in enumerate(opts):
            dg = pricer.batch_diag(i)
            bound = dg["err_est"] * dg["kappa"]
            want = s0[i] if s0[i] != 0 or bound <= g["tol"] else 1
            print(f"  N={N} R={R} option {i} d={o['d']} status {s0[i]} -> {s1[i]} bound {bound:.2e}", flush=True)
            assert s1[i] == want
            if s1[i] == 0:
                n_cert += 1
                ref = F.dense_price(o, N, grids[i][:, 0], grids[i][:, 1])
                assert abs(p1[i] / ref - 1) <= g["tol"]
    assert n_cert > 0
    for bad in (dict(g, certify=2), dict(g, certify=1, n_err_samples=-1)):
        with pytest.raises(ttfp.TTFPError):
            pricer.price_batch(opts[:1], bad)
