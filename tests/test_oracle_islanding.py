"""Pins for the oracle's islanding check (Section II.B.3).

Independent references: SciPy's connected-components routine, closed forms
for trees, cycles and complete graphs, and a Tarjan bridge search written
here (bridges are exactly the branches whose single outage islands)."""
import itertools

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from oracle import islanding


def _scipy_count(n, f, t, on):
    m = coo_matrix((np.ones(int(on.sum())), (f[on], t[on])), shape=(n, n))
    return connected_components(m, directed=False)[0]


def _bridges(n, f, t):
    adj = [[] for _ in range(n)]
    for k, (a, b) in enumerate(zip(f, t)):
        adj[a].append((b, k))
        adj[b].append((a, k))
    disc = [-1] * n
    low = [0] * n
    out = set()
    timer = [0]

    def dfs(u, pe):
        disc[u] = low[u] = timer[0]
        timer[0] += 1
        for v, k in adj[u]:
            if k == pe:
                continue
            if disc[v] < 0:
                dfs(v, k)
                low[u] = min(low[u], low[v])
                if low[v] > disc[u]:
                    out.add(k)
            else:
                low[u] = min(low[u], disc[v])

    for s in range(n):
        if disc[s] < 0:
            dfs(s, -1)
    return out


def _random_graph(rng, n, m):
    edges = set()
    for k in range(1, n):
        edges.add((int(rng.integers(0, k)), k))
    while len(edges) < m:
        a, b = sorted(rng.choice(n, 2, replace=False))
        edges.add((int(a), int(b)))
    e = np.array(sorted(edges))
    return e[:, 0], e[:, 1]


@pytest.mark.parametrize("seed", range(6))
def test_bfs_matches_scipy_on_every_n1_n2(seed):
    rng = np.random.default_rng(seed)
    n, m = 12, 15
    f, t = _random_graph(rng, n, m)
    for i, j in itertools.combinations(range(m), 2):
        on = np.ones(m, bool)
        on[[i, j]] = False
        lab, cnt = islanding.components_bfs(n, f, t, on)
        assert cnt == _scipy_count(n, f, t, on)
        # labels are the minimum bus id of each component
        for r in np.unique(lab):
            assert r == np.flatnonzero(lab == r).min()


def test_tree_every_branch_islands():
    n = 9
    f = np.array([0, 0, 1, 1, 2, 3, 5, 6])
    t = np.array([1, 2, 3, 4, 5, 6, 7, 8])
    for k in range(len(f)):
        on = np.ones(len(f), bool)
        on[k] = False
        assert islanding.components_bfs(n, f, t, on)[1] == 2


def test_cycle_closed_form():
    n = 7
    f = np.arange(n)
    t = (np.arange(n) + 1) % n
    for k in range(n):
        on = np.ones(n, bool)
        on[k] = False
        assert islanding.components_bfs(n, f, t, on)[1] == 1
    for i, j in itertools.combinations(range(n), 2):
        on = np.ones(n, bool)
        on[[i, j]] = False
        assert islanding.components_bfs(n, f, t, on)[1] == 2


def test_complete_graph_never_islands_under_n2():
    n = 5
    pairs = np.array(list(itertools.combinations(range(n), 2)))
    f, t = pairs[:, 0], pairs[:, 1]
    m = len(f)
    for i, j in itertools.combinations(range(m), 2):
        on = np.ones(m, bool)
        on[[i, j]] = False
        assert islanding.components_bfs(n, f, t, on)[1] == 1


@pytest.mark.parametrize("seed", range(4))
def test_n1_islanding_set_equals_bridges(seed):
    rng = np.random.default_rng(100 + seed)
    n, m = 20, 24
    f, t = _random_graph(rng, n, m)
    br = _bridges(n, f, t)
    for k in range(m):
        on = np.ones(m, bool)
        on[k] = False
        cnt = islanding.components_bfs(n, f, t, on)[1]
        assert (cnt > 1) == (k in br)


def test_n2_islands_monotone_over_n1():
    rng = np.random.default_rng(7)
    n, m = 15, 18
    f, t = _random_graph(rng, n, m)
    for i, j in itertools.combinations(range(m), 2):
        on1 = np.ones(m, bool)
        on1[i] = False
        on2 = on1.copy()
        on2[j] = False
        assert (islanding.components_bfs(n, f, t, on2)[1]
                >= islanding.components_bfs(n, f, t, on1)[1])


def test_main_island_largest_capacity_and_tie_rule():
    label = np.array([0, 0, 0, 3, 3, 5])
    gen_bus = np.array([1, 3, 4, 5])
    on = np.ones(4, bool)
    assert islanding.main_island(label, gen_bus, on, np.array([1.0, 0.6, 0.6, 0.5])) == 3
    assert islanding.main_island(label, gen_bus, on, np.array([1.2, 0.6, 0.6, 0.5])) == 0
    # tie -> lowest bus id
    assert islanding.main_island(label, gen_bus, on, np.array([1.0, 0.5, 0.5, 0.5])) == 0
    # reference falls back to the lowest-index generator of the island
    assert islanding.island_reference(label, 3, 0, gen_bus, on) == 3
    assert islanding.island_reference(label, 0, 2, gen_bus, on) == 2


# --- N-3 rows (three outaged branches) ---------------------------------------

def _n3_islands(nb, edges, rows):
    from oracle import islanding
    br_f = np.array([e[0] for e in edges])
    br_t = np.array([e[1] for e in edges])
    out = []
    for row in rows:
        on = np.ones(len(edges), bool)
        on[[k for k in row if k >= 0]] = False
        out.append(islanding.components_bfs(nb, br_f, br_t, on)[1])
    return np.array(out)


def test_n3_closed_forms():
    """Cycle C_n: any three branches out leave exactly 3 paths; a tree: 4
    components; K_6 (edge connectivity 5) never islands under three
    outages."""
    from inputs import contingencies
    n = 9
    cyc = [(k, (k + 1) % n) for k in range(n)]
    rows = contingencies.n3(np.arange(len(cyc)))
    assert len(rows) == 84
    assert np.all(_n3_islands(n, cyc, rows) == 3)
    rng = np.random.default_rng(4)
    tree = [(k, int(rng.integers(0, k))) for k in range(1, 10)]
    assert np.all(_n3_islands(10, tree, contingencies.n3(np.arange(len(tree)))) == 4)
    k6 = [(a, b) for a in range(6) for b in range(a + 1, 6)]
    assert np.all(_n3_islands(6, k6, contingencies.n3(np.arange(len(k6)))) == 1)


def test_n3_enumeration():
    from inputs import contingencies
    from math import comb
    rows = contingencies.n3(np.arange(12))
    assert len(rows) == comb(12, 3)
    assert np.all(rows[:, 0] < rows[:, 1]) and np.all(rows[:, 1] < rows[:, 2])
    assert len({tuple(r) for r in rows}) == len(rows)
    # lexicographic order
    assert [tuple(r) for r in rows] == sorted(tuple(r) for r in rows)


def test_n3_pruning_rule():
    """A triple is pruned exactly when a screened single or pair inside it is
    severe; unscreened subsets prune nothing; N-1 rows are never pruned."""
    from oracle import screen
    sub = np.array([[0, -1], [1, -1], [2, -1], [0, 1], [0, 2], [1, 2], [3, 4]])
    sev = np.array([0, 0, 0, 1, 0, 0, 0])
    rows = np.array([[0, 1, 5], [0, 2, 5], [1, 2, 6], [3, 4, 5], [5, 6, 7], [0, 1, -1],
                     [2, -1, -1], [0, 2, -1]])
    assert screen.n3_prune(rows, sub, sev).tolist() == [False, True, True, True, True, True,
                                                        True, True]
    sev = np.array([0, 0, 1, 0, 0, 0, 1])       # single 2 and pair (3, 4) severe
    assert screen.n3_prune(rows, sub, sev).tolist() == [True, False, False, False, True, True,
                                                        True, False]
