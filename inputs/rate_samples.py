"""Seeded failure-rate samples for the Monte-Carlo analysis of the Risk
Index (random numbers only; none of the method's arithmetic).

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
