"""Network model: pi-branch admittances, bus admittance matrix, post-contingency
subsystem (Section II.B.3 step 1: the numerical model of the network in its
post-contingency state).

Branch model (standard pi model): series admittance y = 1/(r + jx), total
charging b split half per end, off-nominal tap t and phase shift phi on the
from side:
    Yff = (y + jb/2) / t^2,  Yft = -y / (t e^{-j phi}),
    Ytf = -y / (t e^{+j phi}), Ytt = y + jb/2.
Bus shunts gs + j bs add to the diagonal.
"""
from __future__ import annotations

import dataclasses
import numpy as np


def branch_admittances(net):
    r, x, b = net["br_r"], net["br_x"], net["br_b"]
    tap = np.where(net["br_tap"] == 0.0, 1.0, net["br_tap"])
    phi = net["br_shift"]
    y = 1.0 / (r + 1j * x)
    tc = tap * np.exp(1j * phi)
    yff = (y + 0.5j * b) / (tap * tap)
    yft = -y / np.conj(tc)
    ytf = -y / tc
    ytt = y + 0.5j * b
    return yff, yft, ytf, ytt


@dataclasses.dataclass
class Subsystem:
    """Compact post-contingency main island.

    ``bus`` lists original bus ids (ascending); every other array is indexed
    compactly.  ``ref`` is the compact index of the angle reference bus.
    """
    bus: np.ndarray
    ref: int
    br: np.ndarray          # original branch ids in service inside the island
    f: np.ndarray           # compact from-bus of each branch
    t: np.ndarray           # compact to-bus
    gen: np.ndarray         # original generator ids in service in the island
    gbus: np.ndarray        # compact bus of each generator
    pd: np.ndarray          # compact per-bus active load (p.u.)
    qd: np.ndarray
    vmin: np.ndarray
    vmax: np.ndarray
    Y: np.ndarray           # dense complex bus admittance (nb x nb)
    Yf: np.ndarray          # dense complex from-end branch matrix (nl x nb)
    Yt: np.ndarray          # dense complex to-end branch matrix (nl x nb)
    rate: np.ndarray        # branch ratings (p.u.), 0 = unconstrained

    @property
    def nb(self):
        return len(self.bus)


def make_subsystem(net, bus_ids, br_on, gen_on, load_on, ref_orig) -> Subsystem:
    """Build the compact island model from masks over the original network."""
    bus_ids = np.asarray(sorted(bus_ids), dtype=np.int64)
    nb = len(bus_ids)
    pos = -np.ones(int(net["n_bus"]), dtype=np.int64)
    pos[bus_ids] = np.arange(nb)

    fr, to = net["br_from"], net["br_to"]
    br = np.flatnonzero(br_on & (pos[fr] >= 0) & (pos[to] >= 0))
    f, t = pos[fr[br]], pos[to[br]]
    yff, yft, ytf, ytt = (a[br] for a in branch_admittances(net))
    nl = len(br)
    Yf = np.zeros((nl, nb), complex)
    Yt = np.zeros((nl, nb), complex)
    rows = np.arange(nl)
    Yf[rows, f] += yff
    Yf[rows, t] += yft
    Yt[rows, f] += ytf
    Yt[rows, t] += ytt
    Cf = np.zeros((nl, nb))
    Ct = np.zeros((nl, nb))
    Cf[rows, f] = 1.0
    Ct[rows, t] = 1.0
    ysh = net["gs"][bus_ids] + 1j * net["bs"][bus_ids]
    Y = Cf.T @ Yf + Ct.T @ Yt + np.diag(ysh)

    gen = np.flatnonzero(gen_on & (pos[net["gen_bus"]] >= 0))
    gbus = pos[net["gen_bus"][gen]]

    pd = np.zeros(nb)
    qd = np.zeros(nb)
    ld = np.flatnonzero(load_on & (pos[net["load_bus"]] >= 0))
    np.add.at(pd, pos[net["load_bus"][ld]], net["pd"][ld])
    np.add.at(qd, pos[net["load_bus"][ld]], net["qd"][ld])

    return Subsystem(bus=bus_ids, ref=int(pos[ref_orig]), br=br, f=f, t=t,
                     gen=gen, gbus=gbus, pd=pd, qd=qd,
                     vmin=net["vmin"][bus_ids].copy(),
                     vmax=net["vmax"][bus_ids].copy(),
                     Y=Y, Yf=Yf, Yt=Yt, rate=net["br_rate"][br].copy())
