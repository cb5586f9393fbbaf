"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws particles and charges; it holds none of the treecode's
arithmetic.  Workload shapes follow the paper's test problems (Sec. IV:
particles uniform in [-1, 1]^3, charges uniform in [-1, 1], targets equal to
sources) plus a Plummer-sphere distribution and a set of independent systems
of log-uniform size for the batched workload.

All draws use numpy's PCG64 generator, so a (recipe, seed) pair always gives
the same arrays on every machine.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 20030183


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_cube(n: int, seed: int, m: int = 1):
    """n positions uniform in [-1, 1]^3 and m charge vectors uniform in [-1, 1].

    Returns (positions (n, 3) float64, charges (m, n) float64)."""
    g = rng(seed)
    pos = g.uniform(-1.0, 1.0, size=(n, 3))
    q = g.uniform(-1.0, 1.0, size=(m, n))
    return pos, q


def plummer_sphere(n: int, seed: int, m: int = 1, scale: float = 1.0, r_max: float = 10.0):
    """n positions from a Plummer (1911) sphere of scale radius `scale`, truncated at
    r_max, by inverse-CDF sampling of the enclosed-mass fraction
    M(<r) = r^3 / (r^2 + a^2)^{3/2}; isotropic directions; charges uniform in [-1, 1]."""
    g = rng(seed)
    u_max = r_max ** 3 / (r_max ** 2 + scale ** 2) ** 1.5
    u = g.uniform(0.0, u_max, size=n)
    # guard the u = 0 draw (probability zero in exact arithmetic)
    u = np.maximum(u, np.finfo(np.float64).tiny)
    r = scale / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    cos_t = g.uniform(-1.0, 1.0, size=n)
    phi = g.uniform(0.0, 2.0 * np.pi, size=n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    pos = np.stack([r * sin_t * np.cos(phi), r * sin_t * np.sin(phi), r * cos_t], axis=1)
    q = g.uniform(-1.0, 1.0, size=(m, n))
    return pos, q


def log_uniform_sizes(count: int, seed: int, lo_exp: float = 4.0, hi_exp: float = 6.0):
    """`count` system sizes floor(10^U(lo_exp, hi_exp))."""
    g = rng(seed)
    return np.floor(10.0 ** g.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)


def sample_indices(n: int, k: int, seed: int):
    """k distinct indices out of range(n), sorted (error sampling)."""
    g = rng(seed)
    k = min(int(k), int(n))
    return np.sort(g.choice(n, size=k, replace=False)).astype(np.int64)


def config_seed(index: int) -> int:
    """Seed of the workload with the given index (0-based)."""
    return BASE_SEED + int(index)


def sample_seed(index: int) -> int:
    return BASE_SEED + int(index) + 1000
