#!/usr/bin/env python3
"""Throughput benchmark of the TT-cross Fourier pricer on one MI355X.

Workload: d=5 call on the max of 5 GBM assets, drawn from the distributions of the
d=5 configuration (vols ~ U[0.1,0.4], S0 ~ U[80,120], T ~ U[0.25,2], Wishart correlation
with 10 degrees of freedom, K=100, r=0.03), Fourier grid N=128 per dimension with the
automatic truncation / contour rule, TT-cross tol 1e-8, max rank 32, complex FP64.
A step prices one batch of such options (all 5 terms of every option advance together
through the batched HIP path). Each step draws a fresh batch from the same distributions.

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


def surrogate_leg(pricer, grid, n_train, tt_rate):
    """Trains the BF16 surrogate ensemble on TT prices (outside any timed region), then times
    its inference on a batch of 65 536 options and reports its gate statistics."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2203_02804_amd.surrogate import Surrogate

    t0 = time.perf_counter()
    train = W.config5_options(n_train, seed=5)
    labels, _ = pricer.price_batch(train, grid)
    t_label = time.perf_counter() - t0
    sur = Surrogate(d=5, n_models=4, max_batch=65536, seed=3)
    t0 = time.perf_counter()
    info = sur.fit(train, labels, steps=1500, batch=1024, lr=2e-3, holdout=0.1)
    t_fit = time.perf_counter() - t0
    log(f"bench: surrogate labels {t_label:.1f} s, training {t_fit:.1f} s, "
        f"holdout median rel err {np.median(info['holdout_rel_err']):.2e}")
    infer = W.config5_options(65536, seed=55)
    X = sur._x(infer)
    for m in range(sur.n_models):
        sur.net.forward(m, X)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        for m in range(sur.n_models):
            sur.net.forward(m, X)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / reps
    mean, spread = sur.predict(infer)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64, help="options per step")
    ap.add_argument("--max-rank", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-train", type=int, default=4096, help="TT-priced training options")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sharding design is "
              f"described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2203_02804_amd as ttfp
    import workloads as W

    _, grid = W.config2()
    grid = dict(grid, max_rank=args.max_rank)
    B = args.batch
    batches = [W.config2_batch(B, seed=2203 + 1000 * s) for s in range(args.warmup + args.steps)]
    pricer = ttfp.Pricer(0)
    log(f"bench: d=5 N=128 R={grid['max_rank']} batch={B} warmup={args.warmup} steps={args.steps}")
    for s in range(args.warmup):
        pricer.price_batch(batches[s], grid)
        log(f"bench: warmup step {s} done")
    torch.cuda.synchronize()
    if not args.no_profile:
        pricer.profile(True)
    status_all = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        prices, status = pricer.price_batch(batches[args.warmup + s], grid)
        status_all.extend(status.tolist())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = B * args.steps / elapsed
    log(f"bench: timed {args.steps} steps in {elapsed:.3f} s -> {value:.1f} options/s")
    prof = pricer.profile_read() if not args.no_profile else {}
    pricer.profile(False)

    # per-option diagnostics of the timed batches (outside the timed region)
    diag_opts = batches[args.warmup][: min(B, 8)]
    evals, kappas, capped, conv, swaps, halves = [], [], 0, 0, [], []
    for o in diag_opts:
        p, ranks, info, rc = pricer.price(o, grid)
        evals.append(info["n_evals"])
        swaps.append(info["maxvol_swaps"])
        halves.append(info["sweeps"])
        kappas.append(info["kappa"])
        capped += int(info["rank_capped"])
        conv += int(info["converged"])
    evals_per_option = sum(evals) / len(evals)

    # every kernel family: launches, device time, algorithmic rate; the dominant one's roofline
    def rate(name, ms, work):
        if ms <= 0 or work <= 0:
            return None
        if name == "fiber":          # bytes written (16 per complex entry)
            return {"bound": "hbm", "achieved": work / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        return {"bound": "alu", "achieved": work / (ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}

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
                    "traffic": None, "avg_launch_ms": ms / max(n_l, 1), "launches": n_l,
                    "work_per_launch": work / max(n_l, 1)}

    plain = None
    if not args.no_plain:
        opts = batches[0][:4]
        pricer.price(opts[0], grid)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for o in opts:
            pricer.price(o, grid)
        torch.cuda.synchronize()
        plain = len(opts) / (time.perf_counter() - tp0)
        log(f"bench: plain single-option path {plain:.1f} options/s")

    surrogate = None
    if not args.no_surrogate:
        surrogate = surrogate_leg(pricer, grid, args.surrogate_train, value)

    base = None
    if not args.no_cpu_baseline:
        base = cpu_baseline(batches[0][0], grid)
        log(f"bench: cpu baseline {base['value']:.3g} options/s ({base['sample']})")

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
        "config": {"workload": "d5 call-on-max, Wishart(10 dof) correlation, N=128, tol 1e-8, "
                               f"max rank {grid['max_rank']}, batched TT-cross",
                   "global_batch": B, "d": 5, "N": 128, "max_rank": grid["max_rank"], "tol": grid["tol"],
                   "parallelism": "none (1 GPU)"},
        "roofline": roofline,
        "cpu_baseline": base,
        "plain_options_per_s": plain,
        "surrogate": surrogate,
        "kernel_ms": breakdown,
        "accuracy": {"sampled_options": len(diag_opts), "converged": conv, "rank_capped": capped,
                     "median_kappa": sorted(kappas)[len(kappas) // 2],
                     "evals_per_option": evals_per_option,
                     "maxvol_swaps_per_option": sum(swaps) / len(swaps),
                     "half_sweeps_per_option": sum(halves) / len(halves),
                     "status_counts": {str(k): status_all.count(k) for k in sorted(set(status_all))}},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
