"""Counter-based generator used to place sample points (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The sampled error estimate of the cross (Sec. IV.B: relative 1-norm error on random grid
points) draws its points on the device from a counter-based generator, so the tests rebuild
the same points here from the generator's published definition: the SplitMix64 output
function of Steele, Lea and Flood (2014), applied to counters,

    f(x) = z3,  z1 = (x + 0x9E3779B97F4A7C15) mod 2^64,
                z2 = (z1 ^ (z1 >> 30)) * 0xBF58476D1CE4E5B9,
                z3' = (z2 ^ (z2 >> 27)) * 0x94D049BB133111EB,  z3 = z3' ^ (z3' >> 31),

and rand(q, a, b, c, n) = ((h >> 32) * n) >> 32 with h = f(f(f(q ^ a) ^ b) ^ c), an index in
[0, n). The seed of term t of an option priced with grid seed s is
s * 0x100000001B3 + t * 0x9E3779B97F4A7C15 + 1 (mod 2^64); coordinate k of sample point p of
that term is rand(seed_t, 7, p, k, N).

Pinned by the generator's published outputs for seed 0 (tests/test_oracle_rng.py).
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(x: int) -> int:
    z = (x + GOLDEN_GAMMA) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def rand_index(q: int, a: int, b: int, c: int, n: int) -> int:
    h = splitmix64(splitmix64(splitmix64((q ^ a) & MASK) ^ b) ^ c)
    return ((h >> 32) * n) >> 32


def term_seed(grid_seed: int, term: int) -> int:
    return (grid_seed * 0x100000001B3 + term * GOLDEN_GAMMA + 1) & MASK


def sample_points(grid_seed: int, term: int, n_points: int, d: int, N: int) -> np.ndarray:
    """Grid multi-indices [n_points, d] of the error-estimate samples of one term."""
    q = term_seed(grid_seed, term)
    out = np.empty((n_points, d), np.int32)
    for p in range(n_points):
        for k in range(d):
            out[p, k] = rand_index(q, 7, p, k, N)
    return out
