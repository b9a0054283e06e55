"""Islanding check (Section II.B.3) and main-island choice (Section II.A).

After the outage, a graph search over the in-service branches finds every
connected subgraph of buses; more than one subgraph means the scenario is
severe.  An isolated bus is a subgraph of its own (the paper counts all
connected subgraphs).  The island carrying the largest in-service generation
capacity is kept as the reference system for the remaining checks; ties go to
the island holding the lowest bus index.
"""
from __future__ import annotations

from collections import deque
import numpy as np


def components_bfs(n_bus, br_from, br_to, br_on):
    """Breadth-first search labelling.

    Returns ``label`` (int array, each bus labelled with the smallest bus id
    in its component) and the number of components.
    """
    adj = [[] for _ in range(n_bus)]
    for k in np.flatnonzero(br_on):
        a, b = int(br_from[k]), int(br_to[k])
        adj[a].append(b)
        adj[b].append(a)
    label = -np.ones(n_bus, dtype=np.int64)
    n_comp = 0
    for s in range(n_bus):          # ascending start => label = min bus id
        if label[s] >= 0:
            continue
        n_comp += 1
        label[s] = s
        q = deque([s])
        while q:
            u = q.popleft()
            for v in adj[u]:
                if label[v] < 0:
                    label[v] = s
                    q.append(v)
    return label, n_comp


def main_island(label, gen_bus, gen_on, pmax):
    """Label of the island with the largest in-service generation capacity
    (sum of Pmax); ties -> the island with the lowest bus id."""
    roots = np.unique(label)        # ascending == ordered by lowest bus id
    best, best_cap = int(roots[0]), -1.0
    for r in roots:
        cap = float(np.sum(pmax[gen_on & (label[gen_bus] == r)]))
        if cap > best_cap:
            best, best_cap = int(r), cap
    return best


def island_reference(label, main, ref_bus, gen_bus, gen_on):
    """Angle reference of the main island: the network's reference bus if it
    lies in the island, else the bus of the lowest-index in-service generator
    in the island; -1 if the island has no generator."""
    if label[ref_bus] == main:
        return int(ref_bus)
    g = np.flatnonzero(gen_on & (label[gen_bus] == main))
    return int(gen_bus[g[0]]) if len(g) else -1
