"""Autotuner for the pricer's launch parameters.

For a workload shape (d, N, max rank) it times every candidate setting of the launch
parameters that leave the result unchanged bit for bit (graph replay or eager launches; the
tile shapes of the basis and interpolation products, 8 or 16 waves per workgroup with 1 or 2 row
panels per wave, and of the
Gram products, one or two tiles per wave; with the
Householder QR selected, the LDS budget of a TSQR workgroup, which sets its leaf and merge
shapes) on a sample batch of options of that shape, and keeps the fastest. Results are stored in
a JSON table keyed by "d{d}-N{N}-R{R}" next to this module and applied with `apply` (the
pricer's `price_batch` applies the entry of its batch's shape when one exists).
"""
from __future__ import annotations

import itertools
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning_table.json")

CANDIDATES = {
    "graph": (0, 1),
    "mm_waves": (8, 16),
    "mm_panels": (1, 2),
    "gram_threads": (512, 1024),
}
TSQR_CANDIDATES = {"tsqr_lds_kb": (48, 76, 152)}      # only with the Householder QR (qr = 1)


def candidates(pricer):
    """The candidate settings for the pricer's current QR choice."""
    c = dict(CANDIDATES)
    if pricer.get_tuning()["qr"] == 1:
        c.update(TSQR_CANDIDATES)
    return c


def key(d, N, R):
    return f"d{d}-N{N}-R{R}"


def load_table(path=TABLE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def tune(pricer, options, grid, reps=2, path=TABLE, save=True):
    """Times every candidate on `options` (one batch) and returns (best setting, timings)."""
    import torch

    timings = []
    saved = pricer.get_tuning()
    cands = candidates(pricer)
    for values in itertools.product(*cands.values()):
        setting = dict(zip(cands.keys(), values))
        pricer.set_tuning(**setting)
        pricer.price_batch(options, grid)            # warm-up (allocation, code objects)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pricer.price_batch(options, grid)
        torch.cuda.synchronize()
        timings.append((setting, (time.perf_counter() - t0) / reps))
    pricer.set_tuning(**{k: saved[k] for k in cands})
    best = min(timings, key=lambda x: x[1])[0]
    if save:
        table = load_table(path)
        d = options[0]["d"]
        table[key(d, grid["N"], grid["max_rank"])] = dict(best, seconds=min(t for _, t in timings),
                                                          batch=len(options))
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best, timings


def apply(pricer, d, N, R, path=TABLE):
    """Applies the stored setting for (d, N, R), if any; returns it (or None)."""
    entry = load_table(path).get(key(d, N, R))
    if entry:
        pricer.set_tuning(**{k: v for k, v in entry.items() if k in CANDIDATES or k in TSQR_CANDIDATES})
    return entry
