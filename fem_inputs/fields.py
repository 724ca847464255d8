"""Seeded random fields.

Each input field draws from its own NumPy PCG64 stream, spawned from a single
base seed with ``SeedSequence(seed).spawn``, in the fixed stream order
mesh, kappa, f, x, mu, lam, u, lam_adj, flatten; adding a field never shifts
the values of another.
"""
from __future__ import annotations

import numpy as np

STREAMS = ("mesh", "kappa", "f", "x", "mu", "lam", "u", "lam_adj", "flatten")
BASE_SEED = 1501


def spawn_streams(seed: int = BASE_SEED) -> dict:
    kids = np.random.SeedSequence(seed).spawn(len(STREAMS))
    return {name: np.random.Generator(np.random.PCG64(k)) for name, k in zip(STREAMS, kids)}


def seeds(seed: int = BASE_SEED) -> dict:
    return spawn_streams(seed)


def field(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    """n iid values uniform in [lo, hi) as float64."""
    return rng.uniform(lo, hi, size=n).astype(np.float64)
