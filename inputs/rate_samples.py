"""Seeded random inputs beside the networks: failure-rate samples for the
Monte-Carlo analysis of the Risk Index and per-request load snapshots for
serving (random numbers only; none of the method's arithmetic).

Each sample multiplies every component's nominal rate by an independent
log-normal factor exp(sigma z - sigma^2 / 2), z ~ N(0, 1), whose mean is 1.
"""
from __future__ import annotations

import numpy as np


def lognormal_rates(lam, n_samples: int, sigma: float = 0.5, seed: int = 325) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = np.asarray(lam, dtype=np.float64)
    z = rng.standard_normal((n_samples, len(lam)))
    return lam[None, :] * np.exp(sigma * z - 0.5 * sigma * sigma)


def load_scales(n_load: int, n_snapshots: int, sigma: float = 0.05, seed: int = 5000) -> np.ndarray:
    """Per-request load snapshots: every load scaled by an independent factor
    N(1, sigma), clipped at 0.05 from below."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.maximum(rng.normal(1.0, sigma, (n_snapshots, n_load)), 0.05)
