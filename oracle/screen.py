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


@dataclasses.dataclass
class ScreenOptions:
    tol: float = 1e-8
    max_it: int = 150
    near_eps: float = 1e-6
    kkt_solve: str = "lu"               # rounding probes of the OPF (tests only)
    row_scale_seed: int | None = None


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


def evaluate(net, outage, opts: ScreenOptions = ScreenOptions(),
             detail=False) -> ScenarioResult:
    """Evaluate one scenario (outage = (i, j), j = -1 for N-1)."""
    br_on, gen_on, load_on = outage_masks(net, outage)
    nb = int(net["n_bus"])
    label, n_isl = islanding.components_bfs(nb, net["br_from"], net["br_to"], br_on)
    main = islanding.main_island(label, net["gen_bus"], gen_on, net["pmax"])
    ref = islanding.island_reference(label, main, int(net["ref_bus"]),
                                     net["gen_bus"], gen_on)
    cause = CAUSE_ISLAND if n_isl > 1 else 0
    near = 0
    nan = float("nan")
    res = ScenarioResult(severe=0, cause=0, opf_status=opf.NOT_RUN, near=0,
                         n_islands=n_isl, opf_iters=0, n_states=0,
                         opf_cost=nan, max_real_eig=nan, min_damping=nan,
                         max_violation=nan, label=label if detail else None)
    in_main = gen_on & (label[net["gen_bus"]] == main)
    if ref < 0 or not np.any(in_main):
        res.cause = cause | CAUSE_OPF
        res.severe = 1
        return res
    bus_ids = np.flatnonzero(label == main)
    sub = network.make_subsystem(net, bus_ids, br_on, gen_on, load_on, ref)
    o = opf.solve_opf(net, sub, opf.OPFOptions(tol=opts.tol, max_it=opts.max_it,
                                               kkt_solve=opts.kkt_solve,
                                               row_scale_seed=opts.row_scale_seed))
    res.opf_status, res.opf_iters = o.status, o.iters
    res.opf_cost, res.max_violation = o.cost, o.max_violation
    if o.iters >= opts.max_it - 2:
        near |= NEAR_OPF
    if detail:
        res.vm, res.va, res.pg, res.qg = o.vm, o.va, o.pg, o.qg
        res.bus, res.gen = sub.bus, sub.gen
    if o.status != opf.CONVERGED:
        cause |= CAUSE_OPF
        if o.status == opf.NUMERICAL:
            cause |= CAUSE_NUMERICAL
    else:
        if o.max_violation > LIMIT_TOL:
            cause |= CAUSE_LIMIT
        if o.max_violation > 0.1 * LIMIT_TOL:
            near |= NEAR_LIMIT          # within a decade of the limit test
        dm = dynamics.DynModel(net, sub, o.vm, o.va, o.pg, o.qg)
        A = dm.state_matrix()
        res.n_states = A.shape[0]
        if not np.all(np.isfinite(A)):
            cause |= CAUSE_NUMERICAL
        else:
            lam = eigen.eigvals(A)
            alpha, zeta = eigen.spectral_summary(lam)
            res.max_real_eig, res.min_damping = alpha, zeta
            if alpha >= 0.0:
                cause |= CAUSE_SSS
            if abs(alpha) <= opts.near_eps:
                near |= NEAR_SSS
            if detail:
                res.eig = lam
    res.cause = cause
    res.near = near
    res.severe = int(cause != 0)
    return res


def screen(net, outages, lam, opts: ScreenOptions = ScreenOptions()):
    """All scenarios in list order, then the Risk Index of every component."""
    results = [evaluate(net, o, opts) for o in np.asarray(outages)]
    n_comp = int(net["n_branch"]) + int(net["n_gen"]) + int(net["n_load"])
    severe = np.array([r.severe for r in results], dtype=np.uint8)
    R = risk.risk_index(outages, severe, lam, n_comp)
    return results, R


RECORD_FIELDS = ("severe", "cause", "opf_status", "near", "n_islands",
                 "opf_iters", "n_states", "opf_cost", "max_real_eig",
                 "min_damping", "max_violation")


def as_table(results):
    """Per-scenario records as a dict of numpy columns."""
    return {k: np.array([getattr(r, k) for r in results]) for k in RECORD_FIELDS}
