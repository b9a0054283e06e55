"""Per-contingency evaluation loop (Section II.A-II.C), one scenario at a time.

For each outage: take the elements out of service, search for islands,
solve the AC OPF on the main island, check its limits, build the linearised
state matrix at the OPF point, take its eigenvalues, and set the binary
severity S = 1 when any criterion fails (OPF non-convergence or limit
violation, small-signal instability, islanding).  After the loop, eq. (3)
gives each component's Risk Index.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import islanding, network, opf, dynamics, eigen, risk

CAUSE_ISLAND, CAUSE_OPF, CAUSE_LIMIT, CAUSE_SSS, CAUSE_NUMERICAL = 1, 2, 4, 8, 16
NEAR_SSS, NEAR_OPF, NEAR_LIMIT = 1, 2, 4
LIMIT_TOL = 1e-6
NEAR_LIMIT_LO, NEAR_LIMIT_HI = 1e-7, 1e-5     # a decade either side of LIMIT_TOL


@dataclasses.dataclass
class ScreenOptions:
    tol: float = 1e-8
    max_it: int = 150
    near_eps: float = 1e-6
    kkt_solve: str = "lu"               # rounding probes of the OPF (tests only)
    row_scale_seed: int | None = None
    perm_seed: int | None = None


@dataclasses.dataclass
class ScenarioResult:
    severe: int
    cause: int
    opf_status: int
    near: int
    n_islands: int
    opf_iters: int
    n_states: int
    opf_cost: float
    max_real_eig: float
    min_damping: float
    max_violation: float
    # detail (not part of the compact record)
    label: np.ndarray = None
    vm: np.ndarray = None
    va: np.ndarray = None
    pg: np.ndarray = None
    qg: np.ndarray = None
    eig: np.ndarray = None
    bus: np.ndarray = None
    gen: np.ndarray = None
    A: np.ndarray = None


def outage_masks(net, outage):
    nl, ng, nd = int(net["n_branch"]), int(net["n_gen"]), int(net["n_load"])
    br_on = np.ones(nl, bool)
    gen_on = np.ones(ng, bool)
    load_on = np.ones(nd, bool)
    for c in outage:
        c = int(c)
        if c < 0:
            continue
        if c < nl:
            br_on[c] = False
        elif c < nl + ng:
            gen_on[c - nl] = False
        else:
            load_on[c - nl - ng] = False
    return br_on, gen_on, load_on


def near_flags(opf_status, opf_iters, max_violation, alpha,
               opts: ScreenOptions = ScreenOptions()):
    """Decisions that lie close to a threshold (reading of the parity rules;
    the paper's tests themselves are exact).

    NEAR_OPF: the OPF converged within two steps of the iteration cap, so a
      solve rounded differently may end at the cap instead.
    NEAR_LIMIT: the largest limit excess of a converged OPF lies within a
      decade either side of the 1e-6 p.u. test (1e-7 < excess <= 1e-5).
    NEAR_SSS: |max Re lambda| <= near_eps.
    Arguments that were not computed are NaN (and raise no flag)."""
    near = 0
    if opf_status == opf.CONVERGED:
        if opf_iters >= opts.max_it - 2:
            near |= NEAR_OPF
        if NEAR_LIMIT_LO < max_violation <= NEAR_LIMIT_HI:
            near |= NEAR_LIMIT
        if abs(alpha) <= opts.near_eps:
            near |= NEAR_SSS
    return near


def classify(n_islands, opf_status, max_violation, alpha, state_finite=True):
    """Cause bits of one scenario (Section II.B).

    ISLAND: more than one island after the outage (II.B.3).
    OPF: the OPF on the main island did not converge, or could not be run
      (no generator in service there); NUMERICAL in addition when it broke
      down numerically (II.B.1: solver failures count as severe).
    LIMIT: a converged OPF whose largest limit excess is above 1e-6 p.u.
      (II.B.1, operational limits violated).
    SSS: an eigenvalue of the state matrix with real part >= 0 (II.B.2; the
      comparison with zero is inclusive).
    NUMERICAL alone: a converged OPF whose state matrix is not finite.
    The scenario is severe (S = 1) iff any bit is set."""
    cause = CAUSE_ISLAND if n_islands > 1 else 0
    if opf_status != opf.CONVERGED:
        cause |= CAUSE_OPF
        if opf_status == opf.NUMERICAL:
            cause |= CAUSE_NUMERICAL
        return cause
    if max_violation > LIMIT_TOL:
        cause |= CAUSE_LIMIT
    if not state_finite:
        cause |= CAUSE_NUMERICAL
    elif alpha >= 0.0:
        cause |= CAUSE_SSS
    return cause


def evaluate(net, outage, opts: ScreenOptions = ScreenOptions(),
             detail=False) -> ScenarioResult:
    """Evaluate one scenario (outage = (i, j), j = -1 for N-1)."""
    br_on, gen_on, load_on = outage_masks(net, outage)
    nb = int(net["n_bus"])
    label, n_isl = islanding.components_bfs(nb, net["br_from"], net["br_to"], br_on)
    main = islanding.main_island(label, net["gen_bus"], gen_on, net["pmax"])
    ref = islanding.island_reference(label, main, int(net["ref_bus"]),
                                     net["gen_bus"], gen_on)
    nan = float("nan")
    res = ScenarioResult(severe=0, cause=0, opf_status=opf.NOT_RUN, near=0,
                         n_islands=n_isl, opf_iters=0, n_states=0,
                         opf_cost=nan, max_real_eig=nan, min_damping=nan,
                         max_violation=nan, label=label if detail else None)
    in_main = gen_on & (label[net["gen_bus"]] == main)
    if ref < 0 or not np.any(in_main):
        res.cause = classify(n_isl, opf.NOT_RUN, nan, nan)
        res.severe = int(res.cause != 0)
        return res
    bus_ids = np.flatnonzero(label == main)
    sub = network.make_subsystem(net, bus_ids, br_on, gen_on, load_on, ref)
    o = opf.solve_opf(net, sub, opf.OPFOptions(tol=opts.tol, max_it=opts.max_it,
                                               kkt_solve=opts.kkt_solve,
                                               row_scale_seed=opts.row_scale_seed,
                                               perm_seed=opts.perm_seed))
    res.opf_status, res.opf_iters = o.status, o.iters
    res.opf_cost, res.max_violation = o.cost, o.max_violation
    if detail:
        res.vm, res.va, res.pg, res.qg = o.vm, o.va, o.pg, o.qg
        res.bus, res.gen = sub.bus, sub.gen
    finite = True
    if o.status == opf.CONVERGED:
        dm = dynamics.DynModel(net, sub, o.vm, o.va, o.pg, o.qg)
        A = dm.state_matrix()
        res.n_states = A.shape[0]
        finite = bool(np.all(np.isfinite(A)))
        if finite:
            lam = eigen.eigvals(A)
            res.max_real_eig, res.min_damping = eigen.spectral_summary(lam)
            if detail:
                res.eig = lam
                res.A = A
    res.cause = classify(n_isl, o.status, o.max_violation, res.max_real_eig, finite)
    res.near = near_flags(o.status, o.iters, o.max_violation, res.max_real_eig, opts)
    res.severe = int(res.cause != 0)
    return res


def screen(net, outages, lam, opts: ScreenOptions = ScreenOptions()):
    """All scenarios in list order, then the Risk Index of every component."""
    results = [evaluate(net, o, opts) for o in np.asarray(outages)]
    n_comp = int(net["n_branch"]) + int(net["n_gen"]) + int(net["n_load"])
    severe = np.array([r.severe for r in results], dtype=np.uint8)
    R = risk.risk_index(outages, severe, lam, n_comp)
    return results, R


CAUSE_PRUNED = 32


def n3_prune(rows, sub_outages, sub_severe):
    """Rows of three ids to solve (True) or to take as severe without solving
    (False): a row is pruned when one of its single components or pairs is
    severe in the screened N-1/N-2 list (sub_outages, sub_severe); reading:
    more outaged elements never make a severe contingency secure.  Singles
    and pairs absent from that list prune nothing; N-1 rows are never
    pruned, N-2 rows only by their singles."""
    severe_sets = set()
    for row, s in zip(np.asarray(sub_outages), np.asarray(sub_severe)):
        ids = frozenset(int(v) for v in row if v >= 0)
        if s and ids:
            severe_sets.add(ids)
    keep = np.ones(len(rows), bool)
    for r, row in enumerate(np.asarray(rows)):
        ids = [int(v) for v in row if v >= 0]
        subs = [frozenset([a]) for a in ids] if len(ids) >= 2 else []
        if len(ids) == 3:
            subs += [frozenset(p) for p in ((ids[0], ids[1]), (ids[0], ids[2]), (ids[1], ids[2]))]
        keep[r] = not any(sb in severe_sets for sb in subs)
    return keep


RECORD_FIELDS = ("severe", "cause", "opf_status", "near", "n_islands",
                 "opf_iters", "n_states", "opf_cost", "max_real_eig",
                 "min_damping", "max_violation")


def as_table(results):
    """Per-scenario records as a dict of numpy columns."""
    return {k: np.array([getattr(r, k) for r in results]) for k in RECORD_FIELDS}
