"""Contingency lists (Section II.A, exhaustive enumeration).

A list is an int32 array of shape [n, 2]; row ``(i, -1)`` is the N-1 outage of
component ``i`` and ``(i, j)`` the N-2 outage of ``i`` and ``j``.  The paper
enumerates ordered pairs (every ``j != i`` for each ``i``); the synthetic
workloads use each unordered pair once.  Both forms are produced here, along
with seeded random lists for serving-style requests.  Pure index logic.
"""
from __future__ import annotations

import numpy as np


def n1_n2(components, ordered: bool = False) -> np.ndarray:
    """All N-1 outages of ``components`` followed by all N-2 pairs.

    Unordered: pairs (a, b) with a before b in ``components`` order,
    lexicographic.  Ordered: for each a, every b != a (the paper's loop).
    """
    c = np.asarray(components, dtype=np.int32)
    m = len(c)
    n1 = np.stack([c, np.full(m, -1, np.int32)], axis=1)
    if ordered:
        a, b = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        keep = a != b
        pairs = np.stack([c[a[keep]], c[b[keep]]], axis=1)
    else:
        a, b = np.triu_indices(m, k=1)
        pairs = np.stack([c[a], c[b]], axis=1)
    return np.concatenate([n1, pairs.astype(np.int32)], axis=0)


def n3(components) -> np.ndarray:
    """Every unordered triple of ``components`` (rows of three ids, a before
    b before c in ``components`` order, lexicographic)."""
    c = np.asarray(components, dtype=np.int32)
    m = len(c)
    if m < 3:
        return np.zeros((0, 3), np.int32)
    out = []
    for a in range(m - 2):
        for b in range(a + 1, m - 1):
            k = np.arange(b + 1, m)
            out.append(np.stack([np.full(len(k), c[a]), np.full(len(k), c[b]), c[k]], axis=1))
    return np.concatenate(out).astype(np.int32)


def random_list(components, n: int, seed: int, p_n1: float = 0.1) -> np.ndarray:
    """``n`` random outages: N-1 with probability ``p_n1``, else a uniform
    random distinct pair."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.asarray(components, dtype=np.int32)
    out = np.full((n, 2), -1, np.int32)
    for k in range(n):
        if rng.random() < p_n1:
            out[k, 0] = c[rng.integers(0, len(c))]
        else:
            a, b = rng.choice(len(c), 2, replace=False)
            out[k] = (c[a], c[b])
    return out


def c4_list(outage_set, n: int = 20000, seed: int = 300) -> np.ndarray:
    """The 300-bus-shaped workload: n seeded random distinct pairs of the
    outage set (branches and generators)."""
    return random_list(outage_set, n, seed, p_n1=0.0)


def stratified_sample(lst: np.ndarray, n: int, seed: int) -> np.ndarray:
    """Indices of a seeded sample: every N-1 row plus random N-2 rows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n1 = np.flatnonzero(lst[:, 1] < 0)
    n2 = np.flatnonzero(lst[:, 1] >= 0)
    k = max(0, min(len(n2), n - len(n1)))
    pick = np.sort(rng.choice(n2, k, replace=False)) if k else n2[:0]
    return np.concatenate([n1, pick])
