"""GPU parity of the individual kernels, through the C ABI, against the oracle."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import fourier as F
from oracle import ttcross as TT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pricer():
    import paper_2203_02804_amd as ttfp
    p = ttfp.Pricer(0)
    yield p
    p.close()


def _check_integrand(pricer, opt, grid, npts, seed, rtol=1e-13):
    ts, grids = F.term_grids(opt, grid["N"], grid.get("L"), grid.get("alpha"))
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = np.array([g[0] for g in grids])
    As = np.array([g[1] for g in grids])
    g2 = dict(grid, L=Ls, alpha=As)       # the oracle's grid, passed explicitly
    for t, term in enumerate(ts):
        N = grid["N"]
        # half the points anywhere on the grid, half near its centre where the integrand is large
        idx = np.concatenate([rng.integers(0, N, size=(npts // 2, opt["d"])),
                              rng.integers(N // 2 - max(N // 16, 1), N // 2 + max(N // 16, 1),
                                           size=(npts - npts // 2, opt["d"]))])
        gpu = pricer.eval_integrand(opt, g2, t, idx)
        ref = F.integrand_at(term, N, Ls[t], As[t], idx)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(gpu - ref)) <= rtol * scale + 1e-300
        assert np.all(np.abs(gpu - ref) <= 10 * rtol * np.abs(ref) + 1e-2 * rtol * scale)


def test_integrand_small(pricer):
    opt, g = W.config1()
    _check_integrand(pricer, opt, g, 300, 1)
    for opt in W.random_small_options(6, seed=7, d_choices=(1, 2, 3)):
        _check_integrand(pricer, opt, W.grid(48), 200, 2)


def test_integrand_full_size_configs(pricer):
    opt, g = W.config2()
    _check_integrand(pricer, opt, g, 4000, 3)
    opt, g = W.config3()        # d = 20: exponents of size ~100, rounding grows with them
    _check_integrand(pricer, opt, g, 2000, 4, rtol=2e-12)


# Tolerances of the two factorisations behind qr_r. Householder TSQR (qr=1) is backward stable
# column by column (errors of a few ulps of each column's norm). The default three-pass shifted
# Cholesky QR (qr=0) perturbs R^H R by its shifts, 10 nc u of the trace per pass, and the three
# passes bring that to about 2e-13 nc relative (1.2e-11 at nc = 68 in a NumPy replay of the
# kernel's arithmetic on these matrices), far below the rank threshold 0.1 tol / sqrt(d - 1)
# (5e-10 at tol 1e-8) that the factor serves.
QR_TOL = {0: 5e-11, 1: 1e-13}


@pytest.fixture(params=[0, 1], ids=["cholqr", "tsqr"])
def qr_mode(request, pricer):
    pricer.set_tuning(qr=request.param)
    yield request.param
    pricer.set_tuning(qr=0)


@pytest.mark.parametrize("m,n", [(1, 1), (7, 3), (64, 12), (300, 36), (1000, 37), (4096, 36), (2500, 68)])
def test_tsqr_r_factor(pricer, qr_mode, m, n):
    rng = np.random.Generator(np.random.PCG64(m * 1000 + n))
    A = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    if n > 3:   # graded columns: singular values spread over many decades
        A = A * np.logspace(0, -12, n)[None, :]
    print(f"qr_r mode {qr_mode} m={m} n={n}", flush=True)
    R = pricer.qr_r(A)
    assert np.allclose(np.tril(R, -1), 0)
    # R^H R = A^H A and |R| agrees with a reference factor up to the unit diagonal phases
    Rn = np.linalg.qr(A, mode="r")
    k = min(m, n)
    ph = np.diag(Rn)[:k] / np.where(np.diag(R)[:k] == 0, 1, np.diag(R)[:k])
    ph = ph / np.where(np.abs(ph) == 0, 1, np.abs(ph))
    Rg = R[:k] * ph[:, None]
    colnorm = np.linalg.norm(A, axis=0)
    err = np.abs(Rg - Rn[:k]) / colnorm[None, :]
    assert np.max(err) < QR_TOL[qr_mode]
    if m < n:
        assert np.allclose(R[m:], 0)


@pytest.mark.parametrize("m,n", [(256, 36), (7168, 36), (8192, 36), (600, 68)])
def test_tsqr_rows_spanning_hundreds_of_decades(pricer, qr_mode, m, n):
    # fibers of the integrand mix rows near its peak with rows deep in its tails (down to
    # 1e-300 and exact zeros); a leaf block may also hold fewer rows than columns (m=256)
    rng = np.random.Generator(np.random.PCG64(m + 7 * n))
    A = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    A *= 10.0 ** (-300.0 * rng.random(m) ** 3)[:, None]
    A[rng.random(m) < 0.05] = 0.0
    A[: m // 3] *= 1e-170                      # whole leaf blocks of tiny rows
    print(f"qr_r graded rows mode {qr_mode} m={m} n={n}", flush=True)
    R = pricer.qr_r(A)
    assert np.all(np.isfinite(R))
    G0 = A.conj().T @ A
    assert np.linalg.norm(R.conj().T @ R - G0) <= QR_TOL[qr_mode] * np.linalg.norm(G0)
    # the diagonal agrees with a reference factor wherever it is resolved
    d0 = np.abs(np.diag(np.linalg.qr(A, mode="r")))
    dg = np.abs(np.diag(R))
    big = d0 > 1e-10 * d0.max()
    assert np.max(np.abs(dg[big] / d0[big] - 1)) < 1e-6


@pytest.mark.parametrize("seed", range(4))
def test_maxvol_tiny_against_exhaustive_search(pricer, seed):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    m, r = int(rng.integers(5, 11)), int(rng.integers(1, 4))
    A = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    delta = 1e-2
    rows, B = pricer.maxvol(A, delta)
    assert len(set(rows.tolist())) == r
    assert np.allclose(B, A @ np.linalg.inv(A[rows]), atol=1e-12)
    assert np.max(np.abs(B)) <= 1 + delta + 1e-12
    vmax = max(abs(np.linalg.det(A[list(s)])) for s in itertools.combinations(range(m), r))
    assert abs(np.linalg.det(A[rows])) >= vmax / ((1 + delta) ** r * r ** (r / 2)) - 1e-12


def test_maxvol_start_when_largest_rows_are_rank_deficient(pricer):
    # the 100 largest rows span only the first half of the columns (exact zeros elsewhere, as
    # when integrand values underflow): the start must still reach a nonsingular, dominant
    # submatrix
    rng = np.random.Generator(np.random.PCG64(77))
    m, r = 600, 8
    A = 1e-2 * (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r)))
    A[:100, : r // 2] = rng.standard_normal((100, r // 2)) + 1j * rng.standard_normal((100, r // 2))
    A[:100, r // 2:] = 0.0
    rows, B = pricer.maxvol(A, 1e-2)
    assert len(set(rows.tolist())) == r and rows.min() >= 0 and rows.max() < m
    assert np.all(np.isfinite(B))
    ref = A @ np.linalg.inv(A[rows])
    assert np.max(np.abs(B - ref)) < 1e-10
    assert np.max(np.abs(B)) <= 1.01 + 1e-10


@pytest.mark.parametrize("m,r", [(64, 8), (1000, 24), (4096, 32), (8192, 64), (300, 1)])
def test_maxvol_dominance(pricer, m, r):
    rng = np.random.Generator(np.random.PCG64(m + r))
    A = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    Q, _ = np.linalg.qr(A)
    rows, B = pricer.maxvol(Q, 1e-2)
    assert len(set(rows.tolist())) == r
    ref = Q @ np.linalg.inv(Q[rows])
    assert np.max(np.abs(B - ref)) < 1e-11
    assert np.max(np.abs(B)) <= 1.01 + 1e-10
    # the oracle's maxvol from the same start reaches the same dominance bound
    _, Bo = TT.maxvol(Q, 1e-2)
    assert np.max(np.abs(Bo)) <= 1.01 + 1e-10
