"""The allocation-free batch entry point against the allocating one.

ttfp_price_batch_noalloc runs the same kernels as ttfp_price_batch with its whole device
workspace in the library's static per-GPU scratch array. Both are called through the C ABI on
the same seeded options (mixed d, payoffs, Greeks on), twice in a row on the allocation-free
side with the second call smaller than the first, so the second runs on the scratch contents the
first left behind. Prices, deltas and vegas must agree to 1e-12 relative (the kernels and their
inputs are the same, so the expected difference is zero); return codes exactly. A batch whose
workspace exceeds the scratch array is refused before any kernel runs.
"""
import numpy as np
import pytest

import paper_2203_02804_amd as ttfp
import workloads as W

pytestmark = pytest.mark.gpu


def _close(a, b, tol=1e-12):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.all(np.abs(a - b) <= tol * np.maximum(np.abs(b), 1e-300))


def _check_same(pricer, opts, grid):
    p0, dl0, vg0, st0 = pricer.price_batch(opts, grid, greeks=True)
    p1, dl1, vg1, st1 = pricer.price_batch(opts, grid, greeks=True, noalloc=True)
    print(f"noalloc: {len(opts)} options, max |dp|/p = {np.max(np.abs(p1 / p0 - 1)):.2e}", flush=True)
    assert np.array_equal(st0, st1)
    assert _close(p1, p0)
    for a, b in zip(dl1, dl0):
        assert _close(a, b)
    for a, b in zip(vg1, vg0):
        assert _close(a, b)
    return p1


def test_noalloc_matches_price_batch_on_two_calls_second_smaller():
    pricer = ttfp.Pricer(0)
    try:
        opts = W.random_small_options(5, seed=71, d_choices=(2, 3))
        grid = W.grid(64, tol=1e-10, max_rank=16, max_sweeps=4)
        print("noalloc call 1: 5 options, d 2..3, N=64, rank 16", flush=True)
        _check_same(pricer, opts, grid)
        small = W.random_small_options(2, seed=72, d_choices=(1, 2))
        grid2 = W.grid(48, tol=1e-9, max_rank=8, max_sweeps=3)
        print("noalloc call 2: 2 options, d 1..2, N=48, rank 8", flush=True)
        _check_same(pricer, small, grid2)
        # the context's own buffers still serve the allocating path afterwards
        p, st = pricer.price_batch(opts, grid)
        assert np.all(np.isfinite(p))
    finally:
        pricer.close()


def test_noalloc_refuses_a_batch_beyond_the_scratch_array():
    pricer = ttfp.Pricer(0)
    try:
        # d = 5, N = 256, rank 64: about 200 MB of workspace per term, beyond the 128 MiB array
        opts = W.config2_batch(1, seed=2203, corr_kind="beta")
        grid = W.grid(256, tol=1e-8, max_rank=64, max_sweeps=2)
        with pytest.raises(ttfp.TTFPError) as e:
            pricer.price_batch(opts, grid, noalloc=True)
        assert e.value.code == ttfp.TTFP_EINVAL
        assert "workspace" in str(e.value)
    finally:
        pricer.close()
