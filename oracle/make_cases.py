"""Build the stored synthetic network cases (inputs to both the oracle and the
GPU path).

Recipe per shape (the raw draws live in ``inputs.netgen``):
  1. draw the network (attempt = 0, 1, ...);
  2. solve the base-case OPF without flow limits (Section II.A step 1: the
     pre-contingency OPF establishes the reference);
  3. set each branch rating to max(1.5 x the larger end flow |S|, 0.5 p.u.)
     (the floor keeps lightly loaded branches from binding after every
     outage; with 0.1 p.u. about half of the 30-bus N-1 outages are
     infeasible, far from the mostly-secure system the paper studies);
  4. re-solve the base case with the ratings and require convergence, no
     islands and small-signal stability; otherwise draw again.

Usage:  python -m oracle.make_cases [shape ...]   (writes inputs/cases/*.npz)
"""
from __future__ import annotations

import os
import sys
import numpy as np

from inputs import netgen
from . import network, opf, dynamics, eigen, islanding

RATE_FLOOR = 0.5
CASE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "inputs", "cases")


def _full_subsystem(net):
    nb, nl = int(net["n_bus"]), int(net["n_branch"])
    ng, nd = int(net["n_gen"]), int(net["n_load"])
    return network.make_subsystem(net, np.arange(nb), np.ones(nl, bool),
                                  np.ones(ng, bool), np.ones(nd, bool),
                                  int(net["ref_bus"]))


def finalize(net):
    """Ratings from the unconstrained base OPF; returns (net, info) or None."""
    nb = int(net["n_bus"])
    _, n_isl = islanding.components_bfs(nb, net["br_from"], net["br_to"],
                                        np.ones(int(net["n_branch"]), bool))
    if n_isl != 1:
        return None
    sub = _full_subsystem(net)
    o = opf.solve_opf(net, sub)
    if o.status != opf.CONVERGED:
        return None
    V = o.vm * np.exp(1j * o.va)
    Sf = V[sub.f] * np.conj(sub.Yf @ V)
    St = V[sub.t] * np.conj(sub.Yt @ V)
    rate = np.maximum(1.5 * np.maximum(np.abs(Sf), np.abs(St)), RATE_FLOOR)
    net = dict(net)
    net["br_rate"] = np.zeros(int(net["n_branch"]))
    net["br_rate"][sub.br] = rate
    sub = _full_subsystem(net)
    o = opf.solve_opf(net, sub)
    if o.status != opf.CONVERGED:
        return None
    A = dynamics.DynModel(net, sub, o.vm, o.va, o.pg, o.qg).state_matrix()
    alpha, zeta = eigen.spectral_summary(eigen.eigvals(A))
    if not alpha < 0.0:
        return None
    return net, dict(base_cost=o.cost, base_iters=o.iters, base_alpha=alpha,
                     base_zeta=zeta)


def build(shape_name, max_attempts=50):
    shape = netgen.SHAPES[shape_name]
    for attempt in range(max_attempts):
        net = netgen.draw_network(shape, attempt=attempt)
        r = finalize(net)
        if r is not None:
            net, info = r
            net["outage_set"] = netgen.outage_components(net, shape.outage_classes)
            for k, v in info.items():
                net[k] = np.float64(v)
            return net
    raise RuntimeError(f"no admissible draw for {shape_name}")


# 118-bus shape with 16 machines replaced by grid-following converters: the
# same network, loads, machines and ratings as c2_118 otherwise.
C3 = dict(name="c3_118", base="c2_118", n_gfl=16, seed=1180)


def build_c3(max_attempts=50):
    base = netgen.load_case(os.path.join(CASE_DIR, C3["base"] + ".npz"))
    for attempt in range(max_attempts):
        net = netgen.convert_to_gfl(base, C3["n_gfl"], C3["seed"], attempt)
        net["name"] = np.array(C3["name"])
        sub = _full_subsystem(net)
        o = opf.solve_opf(net, sub)
        if o.status != opf.CONVERGED:
            continue
        A = dynamics.DynModel(net, sub, o.vm, o.va, o.pg, o.qg).state_matrix()
        alpha, zeta = eigen.spectral_summary(eigen.eigvals(A))
        if alpha < 0.0:
            net["base_alpha"] = np.float64(alpha)
            net["base_zeta"] = np.float64(zeta)
            return net
    raise RuntimeError("no admissible converter draw")


def main(argv):
    names = argv or list(netgen.SHAPES) + [C3["name"]]
    if C3["name"] in names:
        names = [n for n in names if n != C3["name"]]
        net = build_c3()
        path = os.path.join(CASE_DIR, C3["name"] + ".npz")
        np.savez(path, **net)
        print(f"{C3['name']}: converter attempt {int(net['gfl_attempt'])} alpha "
              f"{float(net['base_alpha']):.6f} zeta {float(net['base_zeta']):.6f} -> {path}")
    os.makedirs(CASE_DIR, exist_ok=True)
    for name in names:
        net = build(name)
        path = os.path.join(CASE_DIR, name + ".npz")
        np.savez(path, **net)
        print(f"{name}: attempt {int(net['attempt'])} base cost "
              f"{float(net['base_cost']):.6f} iters {int(net['base_iters'])} "
              f"alpha {float(net['base_alpha']):.6f} -> {path}")


if __name__ == "__main__":
    main(sys.argv[1:])
