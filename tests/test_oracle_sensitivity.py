"""Scenarios of the 118-bus-shaped list whose OPF outcome rounding decides.

On some post-contingency OPFs (infeasible or nearly so) the interior-point
path wanders for dozens of steps before it settles or its barrier blows up,
and whether it converges depends on the last bits of the Newton solves.
Pinned here on the oracle alone: for every scenario listed in
tests/golden/c2_118_rounding_probes.json (written by
find_rounding_probes.py, which calls only the oracle), solving the same Newton
systems by an exact reformulation (Householder QR, power-of-two row scaling
before the LU, or a symmetric permutation of the system) changes

  outcome  whether the OPF converges (so the severity, Section II.B.1);
  path     the iteration count by more than two, both converged;
  kind     the kind of failure, iteration cap or divergence, both failed.

This is what entitles the full-list parity test to accept a disagreement on
exactly these scenarios and on no other.

The oracle's BLAS runs single-threaded here, as when the stored records were
written (threaded BLAS sums in another order and is itself such a
perturbation).
"""
import json
import os
import warnings
from multiprocessing import get_context

import numpy as np
import pytest

from helpers import GOLDEN, load_case, load_golden

PROBES = os.path.join(GOLDEN, "c2_118_rounding_probes.json")


def _listed():
    data = json.load(open(PROBES))
    return [(what, int(i), tuple(v["outage"]), v["probe"])
            for what in ("outcome", "path", "kind") for i, v in data.get(what, {}).items()]


def _evaluate(args):
    outage, probe = args
    from threadpoolctl import threadpool_limits
    from oracle import screen
    warnings.simplefilter("ignore")
    with threadpool_limits(1):
        r = screen.evaluate(load_case("c2_118"), np.array(outage),
                            screen.ScreenOptions(**probe))
    return r.opf_status, r.opf_iters, r.severe, r.n_islands


@pytest.fixture(scope="module")
def evaluated():
    cases = _listed()
    jobs = [(o, {}) for _, _, o, _ in cases] + [(o, p) for _, _, o, p in cases]
    with get_context("fork").Pool(min(8, len(os.sched_getaffinity(0)))) as pool:
        out = pool.map(_evaluate, jobs)
    n = len(cases)
    return {(w, i): (out[k], out[n + k]) for k, (w, i, _, _) in enumerate(cases)}


def test_list_is_not_empty():
    kinds = {w for w, *_ in _listed()}
    assert {"outcome", "path", "kind"} <= kinds


@pytest.mark.parametrize("what,idx,outage,probe", _listed())
def test_outcome_changes_under_exact_reformulation(evaluated, what, idx, outage, probe):
    g = load_golden("c2_118_full")
    assert tuple(g["outages"][idx]) == outage
    (st, it, sev, isl), (st2, it2, sev2, isl2) = evaluated[(what, idx)]
    # the plain oracle reproduces the stored record
    assert st == g["opf_status"][idx] and it == g["opf_iters"][idx] and sev == g["severe"][idx]
    assert isl == isl2 == g["n_islands"][idx]
    if what == "outcome":
        assert (st == 0) != (st2 == 0)
        assert sev != sev2 or isl > 1
    elif what == "path":
        assert st == st2 == 0 and abs(it - it2) > 2
    else:
        assert st not in (0, 3) and st2 not in (0, 3) and st != st2
        assert sev == sev2 == 1


def test_permutation_probe_is_exact_on_a_small_system():
    """The permutation probe solves the same system: on a well-conditioned
    case its iterates agree with the plain LU to rounding."""
    from oracle import screen
    net = load_case("c1_30")
    a = screen.evaluate(net, np.array([-1, -1]))
    b = screen.evaluate(net, np.array([-1, -1]), screen.ScreenOptions(perm_seed=3))
    assert a.opf_status == b.opf_status == 0
    assert abs(a.opf_cost - b.opf_cost) < 1e-9 * abs(a.opf_cost)
    assert abs(a.opf_iters - b.opf_iters) <= 1
