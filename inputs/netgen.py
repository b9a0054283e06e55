"""Seeded synthetic power networks shaped like the paper's test systems.

The paper evaluates the IEEE 118-bus system (Section IV); its data are not
available here, so every network is drawn from a seeded recipe with the same
shape (bus, branch, generator and load counts).  This module only draws random
numbers: it holds none of the screening method's arithmetic.  Line ratings,
which depend on a base-case power flow, are added afterwards by the oracle's
case builder and stored with the network.

Draw order (numpy PCG64 seeded with ``[seed, attempt]``):
  1. topology: random recursive tree, then extra non-duplicate edges that
     first cover leaves until ``n_pendant`` pendant buses remain;
  2. branch parameters x, r/x, b;
  3. load buses, P, power factor;
  4. generator buses, capacity weights, cost coefficients;
  5. machine parameters (machine base, converted to system base);
  6. failure rates of every component (branches, generators, loads).
"""
from __future__ import annotations

import dataclasses
import numpy as np

# dyn[:, k] column meaning (system base, seconds, per-unit)
DYN_COLS = ("H", "D", "Xd", "Xq", "Xdp", "Xqp", "Td0p", "Tq0p", "Rs",
            "KA", "TA", "R", "Tg", "Tt")
N_DYN = len(DYN_COLS)


@dataclasses.dataclass(frozen=True)
class NetShape:
    name: str
    n_bus: int
    n_branch: int
    n_gen: int
    n_load: int
    seed: int
    n_pendant: int          # pendant (degree-1) buses left uncovered
    outage_classes: tuple   # which component classes are outaged
    load_scale: float = 1.0  # factor on the drawn loads (P and Q)


SHAPES = {
    # 30-bus network: all branch N-1 and N-2 outages
    "c1_30": NetShape("c1_30", 30, 41, 6, 20, 30, 2, ("branch",)),
    # 118-bus-shaped network: every branch, generator and load outaged
    "c2_118": NetShape("c2_118", 118, 186, 54, 99, 118, 6,
                       ("branch", "gen", "load")),
    # 300-bus-shaped network: random N-2 outages of branches and generators;
    # 18 pendant buses make about 8% of random branch/generator pairs island
    # (loads drawn at half the 30- and 118-bus range: with the full range the
    # longer electrical distances of a 300-bus random tree leave the base
    # case infeasible)
    "c4_300": NetShape("c4_300", 300, 411, 69, 200, 300, 18, ("branch", "gen"), 0.5),
}


def _topology(rng, nb, nl, n_pendant):
    edges = []
    present = set()
    deg = np.zeros(nb, dtype=np.int64)
    for k in range(1, nb):
        p = int(rng.integers(0, k))
        edges.append((p, k))
        present.add((p, k))
        deg[p] += 1
        deg[k] += 1
    n_extra = nl - (nb - 1)
    if n_extra < 0:
        raise ValueError("n_branch must be >= n_bus - 1")
    tries = 0
    while len(edges) < nl:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place extra edges")
        leaves = np.flatnonzero(deg == 1)
        if len(leaves) > n_pendant:
            a = int(leaves[rng.integers(0, len(leaves))])
        else:
            a = int(rng.integers(0, nb))
        leaves = np.flatnonzero(deg == 1)
        if len(leaves) > n_pendant + 1:
            b = int(leaves[rng.integers(0, len(leaves))])
        else:
            b = int(rng.integers(0, nb))
        if a == b:
            continue
        e = (min(a, b), max(a, b))
        if e in present:
            continue
        present.add(e)
        edges.append(e)
        deg[a] += 1
        deg[b] += 1
    e = np.array(edges, dtype=np.int32)
    return e[:, 0].copy(), e[:, 1].copy()


def draw_network(shape: NetShape, attempt: int = 0, base_mva: float = 100.0,
                 f_hz: float = 60.0) -> dict:
    """Draw one network of the given shape; returns a dict of numpy arrays.

    ``br_rate`` is left at 0 (unconstrained); the case builder sets it.
    """
    rng = np.random.Generator(np.random.PCG64([shape.seed, attempt]))
    nb, nl, ng, nd = shape.n_bus, shape.n_branch, shape.n_gen, shape.n_load

    br_from, br_to = _topology(rng, nb, nl, shape.n_pendant)

    br_x = rng.uniform(0.02, 0.3, nl)
    br_r = br_x * rng.uniform(0.1, 0.4, nl)
    br_b = rng.uniform(0.0, 0.05, nl)

    load_bus = np.sort(rng.choice(nb, nd, replace=False)).astype(np.int32)
    pd = rng.uniform(0.1, 1.0, nd) * shape.load_scale
    pf = rng.uniform(0.9, 0.98, nd)
    qd = pd * np.tan(np.arccos(pf))

    gen_bus = np.sort(rng.choice(nb, ng, replace=False)).astype(np.int32)
    u = rng.uniform(0.5, 1.5, ng)
    pmax = 1.5 * pd.sum() * u / u.sum()
    pmin = np.zeros(ng)
    qmax = 1.0 * pmax
    qmin = -0.5 * pmax
    c2 = rng.uniform(0.01, 0.1, ng)

    # machine parameters on machine base S_m = 1.2 * Pmax (p.u. of system)
    sm = 1.2 * pmax
    H = rng.uniform(2.5, 6.0, ng)
    D = np.full(ng, 2.0)
    Xd = rng.uniform(1.2, 1.8, ng)
    Xq = 0.9 * Xd
    Xdp = rng.uniform(0.2, 0.35, ng)
    Xqp = rng.uniform(0.4, 0.7, ng)
    Td0p = rng.uniform(5.0, 8.0, ng)
    Tq0p = rng.uniform(0.5, 1.0, ng)
    Rs = np.zeros(ng)
    KA = rng.uniform(50.0, 200.0, ng)
    TA = rng.uniform(0.02, 0.05, ng)
    R = np.full(ng, 0.05)
    Tg = rng.uniform(0.2, 0.5, ng)
    Tt = rng.uniform(0.3, 0.6, ng)
    dyn = np.stack([H * sm, D * sm, Xd / sm, Xq / sm, Xdp / sm, Xqp / sm,
                    Td0p, Tq0p, Rs / sm, KA, TA, R / sm, Tg, Tt], axis=1)

    n_comp = nl + ng + nd
    lam = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), n_comp))

    ref_bus = int(gen_bus[int(np.argmax(pmax))])
    return dict(
        name=np.array(shape.name),
        n_bus=np.int32(nb), n_branch=np.int32(nl), n_gen=np.int32(ng),
        n_load=np.int32(nd), ref_bus=np.int32(ref_bus),
        base_mva=np.float64(base_mva), f_hz=np.float64(f_hz),
        vmin=np.full(nb, 0.90), vmax=np.full(nb, 1.10),
        gs=np.zeros(nb), bs=np.zeros(nb),
        br_from=br_from, br_to=br_to, br_r=br_r, br_x=br_x, br_b=br_b,
        br_rate=np.zeros(nl), br_tap=np.ones(nl), br_shift=np.zeros(nl),
        gen_bus=gen_bus, gen_kind=np.zeros(ng, dtype=np.int32),
        pmin=pmin, pmax=pmax, qmin=qmin, qmax=qmax,
        c2=c2, c1=np.zeros(ng), c0=np.zeros(ng), dyn=dyn,
        load_bus=load_bus, pd=pd, qd=qd, lam=lam,
        attempt=np.int32(attempt),
    )


# converter parameter row (system base); the remaining dyn columns are unused
GFL_COLS = ("Kpp", "Kip", "Kpc", "Kic", "Lf", "Rf", "Cdc", "Kpdc", "Kidc", "Vdc0")


def convert_to_gfl(net: dict, n_gfl: int, seed: int, attempt: int = 0) -> dict:
    """Turn the n_gfl lowest-index synchronous generators that are not at the
    reference bus into grid-following converters with seeded gains.

    Gains are drawn on the converter base S_c = 1.2 Pmax and converted to
    the system base (impedance-like gains divide by S_c, admittance-like and
    energy-like ones multiply by it; the PLL gains are base-free):
      PLL Kpp ~ U(0.05, 0.15), Kip ~ U(1, 3); current PI Kpc ~ U(0.3, 0.6),
      Kic ~ U(5, 15); filter Lf ~ U(0.1, 0.2), Rf ~ U(0.005, 0.02); DC link
      Cdc ~ U(0.05, 0.1) s, DC-voltage PI Kpdc ~ U(1, 3), Kidc ~ U(10, 30),
      Vdc0 = 1."""
    rng = np.random.Generator(np.random.PCG64([seed, attempt]))
    net = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in net.items()}
    ref = int(net["ref_bus"])
    cand = [g for g in range(int(net["n_gen"])) if int(net["gen_bus"][g]) != ref][:n_gfl]
    cand = np.array(cand, dtype=np.int64)
    m = len(cand)
    sc = 1.2 * net["pmax"][cand]
    Kpp = rng.uniform(0.05, 0.15, m)
    Kip = rng.uniform(1.0, 3.0, m)
    Kpc = rng.uniform(0.3, 0.6, m)
    Kic = rng.uniform(5.0, 15.0, m)
    Lf = rng.uniform(0.1, 0.2, m)
    Rf = rng.uniform(0.005, 0.02, m)
    Cdc = rng.uniform(0.05, 0.1, m)
    Kpdc = rng.uniform(1.0, 3.0, m)
    Kidc = rng.uniform(10.0, 30.0, m)
    rows = np.stack([Kpp, Kip, Kpc / sc, Kic / sc, Lf / sc, Rf / sc, Cdc * sc, Kpdc * sc,
                     Kidc * sc, np.ones(m)], axis=1)
    dyn = np.ones((m, N_DYN))
    dyn[:, :len(GFL_COLS)] = rows
    net["gen_kind"] = net["gen_kind"].astype(np.int32).copy()
    net["gen_kind"][cand] = 1
    net["dyn"][cand] = dyn
    net["gfl_attempt"] = np.int32(attempt)
    return net


def outage_components(net: dict, classes) -> np.ndarray:
    """Component ids eligible for outage.

    Component id convention: [0, n_branch) branches, then generators, then
    loads.
    """
    nl, ng, nd = int(net["n_branch"]), int(net["n_gen"]), int(net["n_load"])
    ids = []
    if "branch" in classes:
        ids.append(np.arange(nl))
    if "gen" in classes:
        ids.append(nl + np.arange(ng))
    if "load" in classes:
        ids.append(nl + ng + np.arange(nd))
    return np.concatenate(ids).astype(np.int32)


def load_case(path) -> dict:
    """Load a stored network case (npz, no pickles)."""
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}
