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
