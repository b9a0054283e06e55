"""Shared test helpers: loading cases/golden records, eigenvalue matching."""
from __future__ import annotations

import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
CASES = os.path.join(ROOT, "inputs", "cases")


def load_case(name):
    from inputs import netgen
    return netgen.load_case(os.path.join(CASES, name + ".npz"))


def load_golden(name):
    with np.load(os.path.join(GOLDEN, name + "_oracle.npz"), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def match_eigs(a, b):
    """Greedy nearest-neighbour matching after sorting by (Re desc, Im desc).
    Returns the largest |a_i - b_j| / max(|a_i|, 1) over matched pairs."""
    a = np.asarray(a, complex)
    b = list(np.asarray(b, complex))
    assert len(a) == len(b)
    order = sorted(range(len(a)), key=lambda i: (-a[i].real, -a[i].imag))
    worst = 0.0
    for i in order:
        bb = np.array(b)
        k = int(np.argmin(np.abs(bb - a[i])))
        worst = max(worst, abs(bb[k] - a[i]) / max(abs(a[i]), 1.0))
        b.pop(k)
    return worst


CAUSE_OPF, CAUSE_LIMIT, CAUSE_SSS, CAUSE_NUMERICAL = 2, 4, 8, 16
NEAR_SSS, NEAR_OPF, NEAR_LIMIT = 1, 2, 4


def outcome_mismatches(g, res, flip_ok=()):
    """Compare per-scenario outcomes of the oracle's records g and the
    device's records res (Section II.B decisions).

    Returns (bad, flips, kind) where
      bad   scenarios whose islands, severity, cause or OPF status disagree
            in a way nothing below explains;
      flips scenarios where one OPF converged and the other did not;
      kind  scenarios where both OPFs failed, one at the iteration cap and
            one by divergence.
    Explained disagreements:
      - a decision next to its threshold on either side (near flags):
        NEAR_OPF explains a converged/not-converged split, NEAR_LIMIT the
        LIMIT bit, NEAR_SSS the SSS bit;
      - an OPF outcome split on a scenario listed in flip_ok (each shown to
        flip in the oracle itself under an exact reformulation of its
        Newton solves);
      - where both OPFs failed, the kind of failure (status MAXIT or
        NUMERICAL and the NUMERICAL cause bit): both are severe for the same
        reason, OPF non-convergence."""
    near = np.asarray(g["near"]).astype(int) | np.asarray(res["near"]).astype(int)
    conv_g, conv_d = g["opf_status"] == 0, res["opf_status"] == 0
    ran_g, ran_d = g["opf_status"] != 3, res["opf_status"] != 3
    flip = ran_g & ran_d & (conv_g != conv_d)
    both_failed = ran_g & ran_d & ~conv_g & ~conv_d
    kind = both_failed & (res["opf_status"] != g["opf_status"])
    flip_ok = np.isin(np.arange(len(flip)), np.asarray(list(flip_ok), dtype=np.int64))
    explained_flip = flip & (((near & NEAR_OPF) > 0) | flip_ok)
    mask = np.full(len(flip), 0xFF)
    mask = np.where((near & NEAR_LIMIT) > 0, mask & ~CAUSE_LIMIT, mask)
    mask = np.where((near & NEAR_SSS) > 0, mask & ~CAUSE_SSS, mask)
    mask = np.where(both_failed, mask & ~CAUSE_NUMERICAL, mask)
    cause_g = np.asarray(g["cause"]).astype(int) & mask
    cause_d = np.asarray(res["cause"]).astype(int) & mask
    # each record's severity is its cause bits being set (S = 1 iff any)
    inconsistent = ((np.asarray(res["severe"]) != 0) != (np.asarray(res["cause"]) != 0))
    bad = ((res["n_islands"] != g["n_islands"]) | (ran_g != ran_d) | inconsistent
           | (flip & ~explained_flip)
           | (~flip & (cause_g != cause_d))
           | (~flip & ~both_failed & (res["opf_status"] != g["opf_status"])))
    return np.flatnonzero(bad), np.flatnonzero(flip), np.flatnonzero(kind)


def rounding_listed(outages, what=("outcome",)):
    """Positions in an outage list whose scenario is listed in
    tests/golden/c2_118_rounding_probes.json under one of `what` (the list is
    keyed by position in the full 118-bus-shaped list; rows are matched by
    outage)."""
    import json
    data = json.load(open(os.path.join(GOLDEN, "c2_118_rounding_probes.json")))
    keys = {tuple(v["outage"]) for w in what for v in data.get(w, {}).values()}
    return [k for k, o in enumerate(np.asarray(outages)) if tuple(int(c) for c in o) in keys]
