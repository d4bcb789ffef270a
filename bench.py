#!/usr/bin/env python3
"""Throughput benchmark of the TT-cross Fourier pricer on one MI355X.

Headline workload: d=5 call on the max of 5 GBM assets with the one-factor correlation
Sigma(beta=0.5) of the paper (Sec. V.B) and the d=5 configuration's other draws (vols ~
U[0.1,0.4], S0 ~ U[80,120], T ~ U[0.25,2], K=100, r=0.03), Fourier grid N=256 per dimension with
the automatic truncation / contour rule, TT-cross tol 1e-8, max rank 64, complex FP64. A step
prices one batch of such options (all 5 terms of every option advance together through the
batched HIP path). The value counts the options whose price lies within 1e-6 of the exact
one-factor price (stored references written by the oracle), per second.

Beside it: the raw rate over all options, the single-option (plain) path, the d=5 Wishart
configuration as literally specified (N=128, max rank 32, rank-capped) with its error against
the dense-grid oracle, the BF16 surrogate's inference rate and gate statistics, and the
dense-grid oracle's rate on the host cores.

Prints one JSON line (metric, value, ...). With --gpus > 1 it exits: this build runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "options priced/sec at ≤1e-6 rel. err (TT plain vs batched vs surrogate), 1 GPU"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6          # FP64 vector (and matrix) peak of MI355X
BF16_PEAK_TFLOPS = 2500.0        # dense BF16 MFMA peak of MI355X


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(opt, grid, budget_s=12.0):
    """The dense-grid oracle timed on a bounded slab of one term's grid, extrapolated to
    the whole option (every term, all N^d points)."""
    from oracle import fourier as F

    N = grid["N"]
    d = opt["d"]
    ts, grids = F.term_grids(opt, N, tol=grid["tol"])
    term, (L, A) = ts[0], grids[0]
    rows_total = N ** (d - 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on a small slab, then run a slab of about budget_s seconds
    rows = 2048
    t0 = time.perf_counter()
    F.dense_term_rows(term, N, L, A, 0, rows, nthreads=threads)
    dt = time.perf_counter() - t0
    rows = int(min(rows_total, max(rows, rows * budget_s / max(dt, 1e-6))))
    t0 = time.perf_counter()
    F.dense_term_rows(term, N, L, A, 0, rows, nthreads=threads)
    dt = time.perf_counter() - t0
    sec_per_option = dt * (rows_total / rows) * len(ts)
    return {"value": 1.0 / sec_per_option, "unit": "options/s", "cores": threads, "kind": "oracle",
            "sample": f"dense-grid sum of term 0 of one option over grid rows [0,{rows}) of {rows_total} "
                      f"({rows * N:.3g} of {N ** d:.3g} points, {dt:.1f} s), extrapolated to {len(ts)} terms x "
                      f"{N}^{d} points"}


def host_cpu():
    """Model name and logical core count of the host (from /proc/cpuinfo)."""
    model, n = None, 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    n += 1
                    model = model or line.split(":", 1)[1].strip()
    except OSError:
        pass
    return {"model": model, "logical_cores": n or os.cpu_count()}


def cpu_ttcross(opt, grid):
    """The same method on the CPU: the oracle's NumPy TT-cross (plain loops around LAPACK / BLAS)
    pricing one option of the workload completely (every term, to its own convergence), with the
    grid, tolerance and rank cap of the GPU run. Its integrand calls go to the oracle's C code."""
    from oracle import fourier as F
    from oracle import ttcross as TT

    N = grid["N"]
    ts, grids = F.term_grids(opt, N, tol=grid["tol"])
    t0 = time.perf_counter()
    total = 0j
    for t, (term, (L, A)) in enumerate(zip(ts, grids)):
        fun = lambda idx, term=term, L=L, A=A: F.integrand_at(term, N, L, A, idx)
        cores, _ = TT.tt_cross(fun, opt["d"], N, max_rank=grid["max_rank"], tol=grid["tol"],
                               max_sweeps=grid["max_sweeps"], seed=t)
        total += F.term_scale(opt, L, N) * TT.tt_contract(cores)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "options/s", "seconds": dt, "price": total.real,
            "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "sample": f"one option, all {len(ts)} terms, N={N}, tol {grid['tol']}, max rank {grid['max_rank']}"}


def book_leg(pricer, n, seed_refs):
    """A slice of the batched book (first n options of the 8 192-option book: d ~ U{2..10}, N in
    {64, 128, 256}, rank cap 32, tol 1e-8) priced with deltas and vegas in one batched call."""
    import numpy as np

    import workloads as W

    book, Ns = W.config4()
    opts = book[:n]
    grids = [W.grid(N, tol=1e-8, max_rank=32, max_sweeps=6) for N in Ns[:n]]
    # the stored oracle references of the book's first options with d <= 4 (their own grids)
    refs = {}
    with open(seed_refs) as f:
        for c in json.load(f)["cases"]:
            if c["corr"] == "wishart" and c["index"] < n:
                refs[c["index"]] = c
                grids[c["index"]] = dict(grids[c["index"]], L=np.array(c["L"]), alpha=np.array(c["alpha"]))
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prices, delta, vega, status = pricer.price_batch(opts, grids, greeks=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rel = {i: abs(prices[i] / c["price"] - 1) for i, c in refs.items()}
    return {"workload": f"first {n} options of the batched book (seed 22030), rank cap 32, tol 1e-8, "
                        f"prices with deltas and vegas",
            "options_per_s": n / dt, "seconds": dt,
            "status_counts": {str(k): int(np.sum(status == k)) for k in sorted(set(status.tolist()))},
            "spot_checks_vs_dense_oracle": {"options": len(rel), "within_1e-6": int(sum(v <= 1e-6 for v in rel.values())),
                                            "max_rel_err_converged": max([rel[i] for i in rel if status[i] == 0],
                                                                         default=None)}}


PAPER_GOLDEN = os.path.join(ROOT, "tests", "golden", "paper_table.json")


def paper_table_leg(pricer):
    """The paper's multi-asset experiment (Sec. V.B, Table I): the call on the minimum in asset
    coordinates with the single-strip transform, Sigma(0.5), N = 50 nodes with the table's spacing,
    shift 5 / d, tol 1e-10, rank cap 64; one option per d, priced alone (ttfp_price), against the
    stored exact one-factor price and, for d <= 4, the stored dense grid sum. Then the bond-dimension
    study (d = 3, beta = 0.2, 0.5, 1): the mean error against the grid sum over 4 seeds per rank cap."""
    import numpy as np
    import torch

    import workloads as W

    with open(PAPER_GOLDEN) as f:
        gold = json.load(f)
    rows = []
    for c in gold["table"]:
        d = c["d"]
        opt, g = W.paper_experiment(d)
        pricer.price(opt, g)                              # first call: allocation
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, ranks, info, rc = pricer.price(opt, g)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        row = {"d": d, "eta": 2 * g["L"] / g["N"], "seconds": dt, "status": int(rc), "max_rank": int(ranks.max()),
               "sweeps": info["sweeps"], "n_evals": info["n_evals"], "r_comp": info["n_evals"] / float(g["N"]) ** d,
               "rel_err_vs_exact": p / c["one_factor"] - 1,
               "eps_trunc_vs_grid_sum": (p / c["dense"] - 1) if "dense" in c else None}
        # the paper's own two-train form: caps D_phi = D_v = 40
        opt2, g2 = W.paper_experiment(d, max_rank=40)
        pricer.price_two_trains(opt2, g2, payoff_rank=40)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p2, rcf, rpay, info2, rc2 = pricer.price_two_trains(opt2, g2, payoff_rank=40)
        torch.cuda.synchronize()
        row["two_trains"] = {"seconds": time.perf_counter() - t0, "status": int(rc2), "D_phi": int(rcf.max()),
                             "D_v": int(rpay.max()), "n_evals": info2["n_evals"],
                             "r_comp": info2["n_evals"] / float(g2["N"]) ** d, "rel_err_vs_exact": p2 / c["one_factor"] - 1,
                             "eps_trunc_vs_grid_sum": (p2 / c["dense"] - 1) if "dense" in c else None}
        rows.append(row)
    bond = {}
    for c in gold["bond"]:
        errs = {}
        for R in (3, 6, 12, 24, 48):
            e = []
            for seed in range(4):
                opt, g = W.paper_experiment(3, c["beta"], max_rank=R, seed=seed)
                p, _, _, _ = pricer.price(opt, g)
                e.append(abs(p / c["dense"] - 1))
            errs[str(R)] = float(np.mean(e))
        bond[str(c["beta"])] = errs
    # the bond-dimension study in the two-train form (D_v = 30, cap D_phi swept)
    bond2 = {}
    for c in gold["bond"]:
        errs = {}
        for D in (2, 4, 8, 12, 16):
            e = []
            for seed in range(4):
                opt, g = W.paper_experiment(3, c["beta"], max_rank=D, seed=seed)
                p, _, _, _, _ = pricer.price_two_trains(opt, g, payoff_rank=30)
                e.append(abs(p / c["dense"] - 1))
            errs[str(D)] = float(np.mean(e))
        bond2[str(c["beta"])] = errs
    return {"workload": "call on the min, Sigma(0.5), r=0.3, sigma=0.5, T=1, S0=K=100, N=50, alpha=5/d, tol 1e-10, "
                        "rank cap 64, single strip", "table": rows,
            "bond_dimension_d3": {"mean_rel_err_vs_grid_sum_by_rank_cap": bond, "seeds": 4,
                                  "two_trains_mean_rel_err_by_D_phi_with_D_v_30": bond2}}


LADDER_GOLDEN = os.path.join(ROOT, "tests", "golden", "ladder.json")


def ladder_leg(pricer, grid):
    """A market ladder from one cross (ttfp_price_ladder): the first option of the d = 5 Sigma(0.5)
    batch at 1024 (S0, K, r) points, against their stored exact one-factor prices. Wall time covers
    the base cross and the contractions; the contraction's dense FP64 products are timed with HIP
    events."""
    import numpy as np
    import torch

    import workloads as W

    with open(LADDER_GOLDEN) as f:
        gold = json.load(f)
    ref = np.asarray(gold["prices"])
    base = W.config2_batch(1, seed=gold["batch_seed"], corr_kind="beta")[0]
    S0, K, r = W.ladder_points(base, len(ref), seed=gold["ladder_seed"])
    pricer.price_ladder(base, grid, S0[:16], K[:16], r[:16])         # first call: allocation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prices, info, rc = pricer.price_ladder(base, grid, S0, K, r)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pricer.profile(True)
    pricer.price_ladder(base, grid, S0, K, r)
    n_l, ms, work = pricer.profile_read()["ladder"]
    pricer.profile(False)
    rel = np.abs(prices / ref - 1)
    return {"workload": "1024-point ladder (spots x U[0.85,1.15] per asset, K U[85,115], r U[0,0.06]) around the "
                        "first d5 Sigma(0.5) option, N=256, tol 1e-8, max rank 64, one cross",
            "points": len(ref), "seconds": dt, "points_per_s": len(ref) / dt, "status": int(rc),
            "within_1e-6": int(np.sum(rel <= 1e-6)), "median_rel_err": float(np.median(rel)),
            "max_rel_err": float(rel.max()),
            "contraction_gemm": {"kernel": "k_ladder_core", "launches": n_l, "ms": ms,
                                 "tflops": work / (ms * 1e-3) / 1e12 if ms > 0 else None,
                                 "frac_fp64_peak": work / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS if ms > 0 else None}}


def surrogate_leg(pricer, n_train, tt_rate):
    """Trains the BF16 surrogate ensemble on TT prices (outside any timed region), then times
    its inference on a batch of 65 536 options and reports its gate statistics. Labels: the
    surrogate workload's options with one-factor correlations, priced by the batched TT path at
    N=256, tol 1e-8, max rank 32 (median label error ~3e-5 on this family)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2203_02804_amd.surrogate import Surrogate

    t0 = time.perf_counter()
    grid = W.grid(256, tol=1e-8, max_rank=32, max_sweeps=6)
    train = W.config5_options(n_train, seed=5, corr_kind="beta")
    labels, _ = pricer.price_batch(train, grid)
    t_label = time.perf_counter() - t0
    sur = Surrogate(d=5, n_models=4, max_batch=65536, seed=3)
    t0 = time.perf_counter()
    info = sur.fit(train, labels, steps=3000, batch=1024, lr=2e-3, holdout=0.1)
    t_fit = time.perf_counter() - t0
    log(f"bench: surrogate labels {t_label:.1f} s, training {t_fit:.1f} s, "
        f"holdout median rel err {np.median(info['holdout_rel_err']):.2e}")
    infer = W.config5_options(65536, seed=55, corr_kind="beta")
    X, cv, scale = sur._device_inputs(infer)
    sur.net.predict(X, cv, scale, sur.factor, 1e-4)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        mean, spread, _ = sur.net.predict(X, cv, scale, sur.factor, 1e-4)   # fused ensemble + gate
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / reps
    mean, spread = mean.double().cpu().numpy(), spread.double().cpu().numpy()
    est = sur.factor * spread / np.abs(mean)
    rate = len(infer) / t_inf
    gates = {}
    for g in (1e-2, 1e-4, 1e-6):
        frac = float(np.mean(est <= g))
        # rows failing the gate are re-priced by the batched TT path
        eff = 1.0 / (1.0 / rate + (1.0 - frac) / tt_rate)
        gates[str(g)] = {"served_fraction": frac, "options_per_s_with_fallback": eff}
    flops = 2.0 * len(infer) * sur.net.n_params * sur.n_models
    return {"inference_options_per_s": rate, "batch": len(infer), "models": sur.n_models,
            "mfma_bf16_tflops": flops / t_inf / 1e12, "mfma_bf16_frac": flops / t_inf / 1e12 / BF16_PEAK_TFLOPS,
            "train_options": n_train, "holdout_median_rel_err": float(np.median(info["holdout_rel_err"])),
            "calibration_factor": sur.factor, "gates": gates}


def copy_calibration(nbytes=1 << 30, reps=3):
    """Plain device-to-device copies of nbytes each: a counter of HBM bytes read or written
    should read nbytes per copy; the ratio scales the same counter on the pricer's kernels."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_copy": nbytes, "copies": reps}), flush=True)


GOLDEN = os.path.join(ROOT, "tests", "golden", "one_factor_config2prime.json")
TRAFFIC = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def kernels_digest():
    """SHA-256 over the kernel source and the host code that picks the launch shapes."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "engine.hip"):
        with open(os.path.join(ROOT, "paper_2203_02804_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (two rocprofv3 --pmc
    runs, FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a plain copy of known size),
    or None when there is none for this kernel or the kernel source has changed since."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    kernels = t.get("kernels", {})
    entry = kernels.get(kernel)
    if entry is None:
        # a templated kernel is listed with its instantiation, e.g. k_interp<8>: the one launched
        # most often
        inst = [v for k, v in kernels.items() if k.startswith(kernel + "<")]
        entry = max(inst, key=lambda v: v.get("dispatches", 0)) if inst else None
    if entry is None or t.get("kernels_sha256") != kernels_digest():
        return None
    return entry["bytes_per_launch"]


def load_refs(seed, n):
    """One-factor reference prices of config2_batch(n, seed, 'beta') from the stored golden file
    (written by tests/golden/make_one_factor_golden.py from the oracle), or None."""
    try:
        with open(GOLDEN) as f:
            refs = json.load(f)["batches"].get(str(seed))
    except OSError:
        return None
    return None if refs is None or len(refs) < n else refs[:n]


def time_batches(pricer, batches, grid, warmup, profile):
    import numpy as np
    import torch

    for s in range(warmup):
        pricer.price_batch(batches[s], grid)
    torch.cuda.synchronize()
    if profile:
        pricer.profile(True)
    prices, status = [], []
    t0 = time.perf_counter()
    for b in batches[warmup:]:
        p, st = pricer.price_batch(b, grid)
        prices.append(p)
        status.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = pricer.profile_read() if profile else {}
    pricer.profile(False)
    return np.concatenate(prices), np.concatenate(status), elapsed, prof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=192,
                    help="options per step (960 work items: the one-workgroup-per-item kernels fill the CUs)")
    ap.add_argument("--N", type=int, default=256, help="nodes per dimension (headline workload)")
    ap.add_argument("--max-rank", type=int, default=64, help="rank cap (headline workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-literal", action="store_true", help="skip the literal Wishart N=128 R=32 line")
    ap.add_argument("--surrogate-train", type=int, default=4096, help="TT-priced training options")
    ap.add_argument("--no-book", action="store_true", help="skip the batched-book leg")
    ap.add_argument("--book", type=int, default=8192, help="options of the batched book in its leg")
    ap.add_argument("--no-cpu-ttcross", action="store_true", help="skip the CPU TT-cross timing")
    ap.add_argument("--no-paper-table", action="store_true", help="skip the paper's call-on-min experiment")
    ap.add_argument("--no-ladder", action="store_true", help="skip the market-ladder leg")
    ap.add_argument("--no-diag", action="store_true",
                    help="skip the per-option diagnostics after the timed region (so that a kernel trace of the "
                         "run holds the batches' launches only)")
    ap.add_argument("--qr", choices=["cholqr", "tsqr", "cholqr2", "cholqr3"], default="cholqr",
                    help="triangular factor of the fibers: shifted Cholesky QR on the matrix cores with passes "
                         "chosen by the rank threshold, Householder TSQR, or two / three Cholesky QR passes")
    ap.add_argument("--mv-rounds", type=int, default=3, help="maxvol refinement rounds after the block start")
    ap.add_argument("--mv-warm", type=int, default=1, choices=(0, 1),
                    help="maxvol starts from the previous same-direction pivots (1) or always by elimination (0)")
    ap.add_argument("--mm-waves", type=int, default=None, choices=(8, 16),
                    help="16-row panels per workgroup of the basis and interpolation products (default: the "
                         "autotuner's stored choice for the workload's shape, else 8)")
    ap.add_argument("--mm-panels", type=int, default=None, choices=(1, 2),
                    help="16-row panels per wave of the basis and interpolation products (default: the autotuner's "
                         "stored choice, else 1)")
    ap.add_argument("--gram-threads", type=int, default=None, choices=(512, 1024),
                    help="threads per Gram workgroup (default: the autotuner's stored choice, else 512)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of a known size (scales the HBM byte counters of a profiler)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): options and terms are "
              f"independent, so a multi-GPU run would split the batch by option; it is not measured here",
              file=sys.stderr)
        sys.exit(2)
    with open(GOLDEN) as f:
        stored = json.load(f)
    if args.batch > stored["batch"]:
        print(f"the stored references cover batches of at most {stored['batch']} options", file=sys.stderr)
        sys.exit(2)
    stored_seeds = sorted(int(s) for s in stored["batches"])

    import numpy as np
    import torch

    import paper_2203_02804_amd as ttfp
    import workloads as W

    B = args.batch
    grid = W.grid(args.N, tol=1e-8, max_rank=args.max_rank, max_sweeps=8)
    # one stored batch per step; more steps than stored batches cycle through them again (every
    # step is priced from scratch, nothing is cached between steps)
    seeds = [stored_seeds[s % len(stored_seeds)] for s in range(args.warmup + args.steps)]
    batches = [W.config2_batch(B, seed=sd, corr_kind="beta") for sd in seeds]
    refs = np.concatenate([load_refs(sd, B) for sd in seeds[args.warmup:]])
    pricer = ttfp.Pricer(0)
    pricer.set_tuning(qr={"cholqr": 0, "tsqr": 1, "cholqr2": 2, "cholqr3": 3}[args.qr], maxvol_rounds=args.mv_rounds,
                      maxvol_warm=args.mv_warm)
    if args.mm_waves is not None or args.gram_threads is not None or args.mm_panels is not None:
        pricer.autotune = False
        if args.mm_waves is not None:
            pricer.set_tuning(mm_waves=args.mm_waves)
        if args.mm_panels is not None:
            pricer.set_tuning(mm_panels=args.mm_panels)
        if args.gram_threads is not None:
            pricer.set_tuning(gram_threads=args.gram_threads)
    log(f"bench: d=5 Sigma(0.5) N={args.N} R={args.max_rank} batch={B} warmup={args.warmup} steps={args.steps}")
    prices, status, elapsed, prof = time_batches(pricer, batches, grid, args.warmup, not args.no_profile)
    launch_tuning = pricer.get_tuning()
    n_opt = B * args.steps
    rel = np.abs(prices / refs - 1.0)
    good = int(np.sum(rel <= 1e-6))
    value = good / elapsed
    log(f"bench: timed {args.steps} steps in {elapsed:.3f} s: {n_opt / elapsed:.2f} options/s, "
        f"{good}/{n_opt} within 1e-6 -> {value:.2f} options/s at <=1e-6")

    # every kernel family: launches, device time, algorithmic rate; the dominant one's roofline
    def rate(name, ms, work):
        if ms <= 0 or work <= 0:
            return None
        if name == "fiber":          # bytes written (16 per complex entry)
            return {"bound": "hbm", "achieved": work / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        # the Gram, transform, basis and interpolation products run on the FP64 matrix cores; the
        # other families are FP64 vector arithmetic (both peaks are 78.6 TFLOP/s on MI355X)
        bound = "mfma" if name in ("gram", "xform", "basis", "interp") else "alu"
        return {"bound": bound, "achieved": work / (ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}

    roofline = None
    breakdown = {}
    for k, (n, ms, work) in prof.items():
        breakdown[k] = {"launches": n, "ms": round(ms, 3)}
        rr = rate(k, ms, work)
        if rr:
            breakdown[k].update({"achieved": rr["achieved"], "unit": rr["unit"], "frac": rr["achieved"] / rr["peak"]})
    if prof:
        dom = max(prof, key=lambda k: prof[k][1])
        n_l, ms, work = prof[dom]
        rr = rate(dom, ms, work)
        roofline = {"kernel": "k_" + dom, "bound": rr["bound"] if rr else None,
                    "achieved": rr["achieved"] if rr else None, "peak": rr["peak"] if rr else None,
                    "unit": rr["unit"] if rr else None, "frac": rr["achieved"] / rr["peak"] if rr else None,
                    "traffic": measured_traffic("k_" + dom), "avg_launch_ms": ms / max(n_l, 1), "launches": n_l,
                    "work_per_launch": work / max(n_l, 1)}

    # per-option diagnostics of two options (outside the timed region)
    diag = []
    for o in ([] if args.no_diag else batches[args.warmup][:2]):
        _, ranks, info, rc = pricer.price(o, grid)
        diag.append(dict(max_rank_reached=int(ranks.max()), n_evals=info["n_evals"], half_sweeps=info["sweeps"],
                         maxvol_swaps=info["maxvol_swaps"], maxvol_full_starts=info["maxvol_full_starts"],
                         kappa=info["kappa"], converged=info["converged"]))

    plain = None
    if not args.no_plain:
        opts = batches[args.warmup][:2]
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        pp = [pricer.price(o, grid)[0] for o in opts]
        torch.cuda.synchronize()
        plain = {"options_per_s": len(opts) / (time.perf_counter() - tp0), "options": len(opts),
                 "max_rel_err": float(np.max(np.abs(np.array(pp) / refs[: len(opts)] - 1)))}
        log(f"bench: plain single-option path {plain['options_per_s']:.2f} options/s")

    literal = None
    if not args.no_literal:
        # the d=5 Wishart configuration as literally specified (N=128, max rank 32): rank-capped
        _, g2 = W.config2()
        lsteps = min(args.steps, 3)
        lb = [W.config2_batch(B, seed=sd) for sd in stored_seeds[: 1 + lsteps]]
        lp, lst, lel, _ = time_batches(pricer, lb, g2, 1, False)
        with open(os.path.join(ROOT, "tests", "golden", "dense_config2.json")) as f:
            dense0 = json.load(f)["cases"][0]["price"]
        p0 = pricer.price_batch(lb[0][:1], g2)[0][0]
        literal = {"workload": "d5 call-on-max, Wishart(10 dof) correlation, N=128, tol 1e-8, max rank 32",
                   "options_per_s": B * lsteps / lel,
                   "status_counts": {str(k): int(np.sum(lst == k)) for k in sorted(set(lst.tolist()))},
                   "option0_rel_err_vs_dense_grid_oracle": float(p0 / dense0 - 1)}
        log(f"bench: literal Wishart N=128 R=32: {literal['options_per_s']:.1f} options/s, option 0 error "
            f"{literal['option0_rel_err_vs_dense_grid_oracle']:.2e} vs the dense oracle")

    surrogate = None
    if not args.no_surrogate:
        surrogate = surrogate_leg(pricer, args.surrogate_train, n_opt / elapsed)

    book = None
    if not args.no_book:
        book = book_leg(pricer, args.book, os.path.join(ROOT, "tests", "golden", "book_slice.json"))
        log(f"bench: book slice {book['options_per_s']:.1f} options/s with Greeks, status {book['status_counts']}")

    ladder = None
    if not args.no_ladder:
        ladder = ladder_leg(pricer, grid)
        log(f"bench: ladder {ladder['points_per_s']:.0f} points/s, {ladder['within_1e-6']}/{ladder['points']} within "
            f"1e-6, contraction {ladder['contraction_gemm']['tflops']:.1f} TFLOP/s")

    paper = None
    if not args.no_paper_table:
        paper = paper_table_leg(pricer)
        log("bench: paper table " + " ".join(f"d={r['d']}:{r['seconds'] * 1e3:.0f}ms/{r['rel_err_vs_exact']:+.1e}"
                                             for r in paper["table"]))

    base = None
    if not args.no_cpu_baseline:
        base = cpu_baseline(batches[args.warmup][0], grid)
        base["host_cpu"] = host_cpu()
        log(f"bench: cpu baseline {base['value']:.3g} options/s ({base['sample']})")
        if not args.no_cpu_ttcross:
            base["same_method_cpu"] = cpu_ttcross(batches[args.warmup][0], grid)
            log(f"bench: cpu TT-cross {base['same_method_cpu']['seconds']:.1f} s per option")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "options/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"d5 call-on-max, one-factor correlation Sigma(0.5) with the d=5 configuration's "
                               f"other draws, N={args.N}, tol 1e-8, max rank {args.max_rank}, batched TT-cross; "
                               f"value counts options within 1e-6 of the one-factor reference",
                   "global_batch": B, "d": 5, "N": args.N, "max_rank": args.max_rank, "tol": 1e-8,
                   "parallelism": "none (1 GPU)", "launch_tuning": launch_tuning},
        "roofline": roofline,
        "cpu_baseline": base,
        "throughput_all_options_per_s": n_opt / elapsed,
        "accuracy": {"options": n_opt, "within_1e-6": good, "median_rel_err": float(np.median(rel)),
                     "p90_rel_err": float(np.quantile(rel, 0.9)), "max_rel_err": float(rel.max()),
                     "converged": int(np.sum(status == 0)),
                     "max_rel_err_converged": float(rel[status == 0].max()) if np.any(status == 0) else None,
                     "sample_diagnostics": diag},
        "plain": plain,
        "literal_config2": literal,
        "book": book,
        "ladder": ladder,
        "paper_table": paper,
        "surrogate": surrogate,
        "kernel_ms": breakdown,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
