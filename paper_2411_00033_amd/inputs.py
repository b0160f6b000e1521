"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the transform: it only draws coefficient
vectors.  The paper's experiments use seeded random coefficients that decay
with the index (Sec. 5.1); here they are standard normal draws z_j from
numpy's PCG64 generator, scaled as f_j = z_j / (j+1)^r.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 2411000


def decaying(n: int, r: float, seed: int, batch: int | None = None) -> np.ndarray:
    """f_j = z_j / (j+1)^r with z_j iid N(0,1); shape (n,) or (batch, n), float64."""
    rng = np.random.default_rng(seed)
    shape = (n,) if batch is None else (batch, n)
    z = rng.standard_normal(shape)
    return z / np.power(np.arange(1, n + 1, dtype=np.float64), r)


def uniform01(n: int, seed: int) -> np.ndarray:
    """Coefficients uniform on [0, 1) (the undecayed r = 0 input of Table 1)."""
    return np.random.default_rng(seed).random(n)


def ragged_sizes(count: int, seed: int, lo: int = 128, hi: int = 262144):
    """Sizes log-uniform in [lo, hi] and directions Bernoulli(1/2), from one stream."""
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    n = np.clip(n, lo, hi)
    direction = (rng.random(count) < 0.5).astype(np.int32)
    return n, direction
