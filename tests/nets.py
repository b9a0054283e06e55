"""Tiny hand-built networks for closed-form pins (test helpers only)."""
from __future__ import annotations

import numpy as np

from inputs import netgen


def base_dyn_row(**kw):
    d = dict(H=4.0, D=2.0, Xd=1.5, Xq=1.4, Xdp=0.3, Xqp=0.5, Td0p=6.0,
             Tq0p=0.8, Rs=0.0, KA=100.0, TA=0.03, R=0.05, Tg=0.3, Tt=0.4)
    d.update(kw)
    return [d[k] for k in netgen.DYN_COLS]


def make_net(n_bus, branches, gens, loads, ref_bus=0, vmin=0.9, vmax=1.1,
             rate=None, base_mva=100.0, f_hz=60.0):
    """branches: list of (f, t, r, x, b); gens: list of dicts with bus,
    pmin, pmax, qmin, qmax, c2, c1 and optional dyn; loads: (bus, pd, qd)."""
    nl, ng, nd = len(branches), len(gens), len(loads)
    br = np.array(branches, dtype=float).reshape(nl, 5)
    net = dict(
        name=np.array("tiny"),
        n_bus=np.int32(n_bus), n_branch=np.int32(nl), n_gen=np.int32(ng),
        n_load=np.int32(nd), ref_bus=np.int32(ref_bus),
        base_mva=np.float64(base_mva), f_hz=np.float64(f_hz),
        vmin=np.full(n_bus, vmin), vmax=np.full(n_bus, vmax),
        gs=np.zeros(n_bus), bs=np.zeros(n_bus),
        br_from=br[:, 0].astype(np.int32), br_to=br[:, 1].astype(np.int32),
        br_r=br[:, 2].copy(), br_x=br[:, 3].copy(), br_b=br[:, 4].copy(),
        br_rate=np.zeros(nl) if rate is None else np.asarray(rate, float),
        br_tap=np.ones(nl), br_shift=np.zeros(nl),
        gen_bus=np.array([g["bus"] for g in gens], np.int32),
        gen_kind=np.zeros(ng, np.int32),
        pmin=np.array([g.get("pmin", 0.0) for g in gens]),
        pmax=np.array([g.get("pmax", 10.0) for g in gens]),
        qmin=np.array([g.get("qmin", -10.0) for g in gens]),
        qmax=np.array([g.get("qmax", 10.0) for g in gens]),
        c2=np.array([g.get("c2", 0.05) for g in gens]),
        c1=np.array([g.get("c1", 0.0) for g in gens]),
        c0=np.zeros(ng),
        dyn=np.array([g.get("dyn", base_dyn_row()) for g in gens], float).reshape(ng, -1),
        load_bus=np.array([l[0] for l in loads], np.int32),
        pd=np.array([l[1] for l in loads], float),
        qd=np.array([l[2] for l in loads], float),
    )
    net["lam"] = np.full(nl + ng + nd, 0.01)
    return net


def full_subsystem(net):
    from oracle import network
    nb, nl = int(net["n_bus"]), int(net["n_branch"])
    ng, nd = int(net["n_gen"]), int(net["n_load"])
    return network.make_subsystem(net, np.arange(nb), np.ones(nl, bool),
                                  np.ones(ng, bool), np.ones(nd, bool),
                                  int(net["ref_bus"]))
