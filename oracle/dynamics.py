"""Linearised state matrix at the OPF operating point (Section II.B.2).

The paper builds the full dynamic model at the OPF point, linearises it and
inspects the eigenvalues of the state matrix; it leaves the device models to
its simulation tool, and its generation units are "generators or converters"
(Section IV).  The oracle uses standard phasor models.

Synchronous generator (kind 0), two-axis model of Sauer and Pai (Power
System Dynamics and Stability), states
  x = [delta, omega, Eq', Ed', Efd, Psv, Pm]
  delta' = ws (omega - 1)
  2H omega' = Pm - Pe - D (omega - 1),  Pe = Ed' Id + Eq' Iq + (Xq' - Xd') Id Iq
  Td0' Eq'' = -Eq' - (Xd - Xd') Id + Efd
  Tq0' Ed'' = -Ed' + (Xq - Xq') Iq
  TA Efd'   = -Efd + KA (Vref - V)                      (first-order AVR)
  Tg Psv'   = -Psv + Pref - (omega - 1)/R                (governor)
  Tt Pm'    = -Pm + Psv                                   (turbine)
stator (algebraic):
  0 = Ed' - V sin(delta - theta) - Rs Id + Xq' Iq
  0 = Eq' - V cos(delta - theta) - Rs Iq - Xd' Id
injection: P = Id V sin(delta-theta) + Iq V cos(delta-theta),
           Q = Id V cos(delta-theta) - Iq V sin(delta-theta).

Grid-following converter (kind 1): a current-controlled source synchronised
by a phase-locked loop, with an L filter and a DC link, states
  x = [theta_p, x_pll, x_id, x_iq, i_d, i_q, v_dc, x_dc]
in the PLL frame (v_d + j v_q = V e^{j(theta - theta_p)}):
  theta_p' = ws (Kpp v_q + Kip x_pll)                  (PLL, drives v_q to 0)
  x_pll'   = v_q
  x_id'    = i_d* - i_d,   i_d* = Kpdc (v_dc - Vdc0) + Kidc x_dc
  x_iq'    = i_q* - i_q,   i_q* = i_q at the operating point
  (Lf/ws) i_d' = Kpc (i_d* - i_d) + Kic x_id - Rf i_d  (current PI with voltage
  (Lf/ws) i_q' = Kpc (i_q* - i_q) + Kic x_iq - Rf i_q   feed-forward, decoupled)
  Cdc v_dc v_dc' = Pdc - (v_d i_d + v_q i_q)           (DC link, constant source)
  x_dc'    = v_dc - Vdc0                               (DC-voltage PI)
injection: the current (i_d + j i_q) e^{j theta_p},
  P = V (i_d cos phi + i_q sin phi), Q = V (i_d sin phi - i_q cos phi),
  phi = theta - theta_p.

Loads are constant impedances at the OPF voltage: P0 (V/V0)^2, Q0 (V/V0)^2;
the network balance is injection - load - V conj(Y V) at every island bus.

Algebraic variables y = [Id, Iq (synchronous machines), theta, V].
Linearisation: A_full = f_x - f_y g_y^{-1} g_x.  The absolute angles leave a
structural zero eigenvalue (a uniform shift of every angle, rotor and PLL, is
an equilibrium).  It is removed by taking angles relative to the first
device's angle state: every other device's angle row minus that one, then
its row and column deleted.
"""
from __future__ import annotations

import numpy as np

from .opf import complex_power_jac

NS_SG = 7       # states per synchronous generator
NS_GFL = 8      # states per grid-following converter
SG, GFL = 0, 1
# dyn row of a converter (system base)
GFL_COLS = ("Kpp", "Kip", "Kpc", "Kic", "Lf", "Rf", "Cdc", "Kpdc", "Kidc", "Vdc0")


class DynModel:
    def __init__(self, net, sub, vm, va, pg, qg):
        kind = np.asarray(net["gen_kind"])[sub.gen]
        if np.any((kind != SG) & (kind != GFL)):
            raise NotImplementedError("device kinds 0 (SG) and 1 (GFL) only")
        self.sub = sub
        self.nb = nb = sub.nb
        self.ws = 2.0 * np.pi * float(net["f_hz"])
        self.kind = kind
        sizes = np.where(kind == SG, NS_SG, NS_GFL)
        self.off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        self.nx = int(sizes.sum())
        self.isg = np.flatnonzero(kind == SG)          # device positions
        self.icv = np.flatnonzero(kind == GFL)
        self.nsg = nsg = len(self.isg)
        self.k = sub.gbus
        self.ksg = sub.gbus[self.isg]
        self.kcv = sub.gbus[self.icv]
        dyn = np.asarray(net["dyn"])[sub.gen]
        # synchronous machines
        p = dyn[self.isg]
        (self.H, self.D, self.Xd, self.Xq, self.Xdp, self.Xqp, self.Td0p,
         self.Tq0p, self.Rs, self.KA, self.TA, self.R, self.Tg,
         self.Tt) = p.T
        # converters
        c = dyn[self.icv][:, :len(GFL_COLS)]
        (self.Kpp, self.Kip, self.Kpc, self.Kic, self.Lf, self.Rf, self.Cdc,
         self.Kpdc, self.Kidc, self.Vdc0) = c.T
        self.P0 = sub.pd.copy()
        self.Q0 = sub.qd.copy()
        self.V0 = vm.copy()
        x = np.zeros(self.nx)
        # --- machine equilibrium from the operating point -------------------
        V = vm * np.exp(1j * va)
        Vg = V[self.ksg]
        I = np.conj((pg[self.isg] + 1j * qg[self.isg]) / Vg)
        EQ = Vg + (self.Rs + 1j * self.Xq) * I
        delta = np.angle(EQ)
        rot = np.exp(-1j * (delta - np.pi / 2))
        Idq = I * rot
        Vdq = Vg * rot
        Id, Iq = Idq.real, Idq.imag
        Vd, Vq = Vdq.real, Vdq.imag
        Edp = Vd + self.Rs * Id - self.Xqp * Iq
        Eqp = Vq + self.Rs * Iq + self.Xdp * Id
        Efd = Eqp + (self.Xd - self.Xdp) * Id
        safe = np.where(self.KA != 0.0, self.KA, 1.0)
        self.Vref = vm[self.ksg] + np.where(self.KA != 0.0, Efd / safe, 0.0)
        Pm = Edp * Id + Eqp * Iq + (self.Xqp - self.Xdp) * Id * Iq
        self.Pref = Pm.copy()
        o = self.off[self.isg]
        for t, v in enumerate([delta, np.ones(nsg), Eqp, Edp, Efd, Pm, Pm]):
            x[o + t] = v
        # --- converter equilibrium: PLL locked (v_q = 0), currents from P, Q
        vk = vm[self.kcv]
        idc = pg[self.icv] / vk
        iqc = -qg[self.icv] / vk
        self.iq_ref = iqc.copy()
        self.Pdc = pg[self.icv].copy()
        o = self.off[self.icv]
        for t, v in enumerate([va[self.kcv], np.zeros(len(o)), self.Rf * idc / self.Kic,
                               self.Rf * iqc / self.Kic, idc, iqc, self.Vdc0,
                               idc / self.Kidc]):
            x[o + t] = v
        self.x0 = x
        self.y0 = np.concatenate([Id, Iq, va, vm])

    # --- residuals --------------------------------------------------------
    def split(self, y):
        nsg, nb = self.nsg, self.nb
        return y[:nsg], y[nsg:2 * nsg], y[2 * nsg:2 * nsg + nb], y[2 * nsg + nb:]

    def sg_states(self, x):
        o = self.off[self.isg]
        return [x[o + t] for t in range(NS_SG)]

    def cv_states(self, x):
        o = self.off[self.icv]
        return [x[o + t] for t in range(NS_GFL)]

    def f(self, x, y):
        Id, Iq, th, v = self.split(y)
        out = np.zeros(self.nx)
        d, w, Eq, Ed, Efd, Psv, Pm = self.sg_states(x)
        Pe = Ed * Id + Eq * Iq + (self.Xqp - self.Xdp) * Id * Iq
        o = self.off[self.isg]
        rows = [self.ws * (w - 1.0),
                (Pm - Pe - self.D * (w - 1.0)) / (2.0 * self.H),
                (-Eq - (self.Xd - self.Xdp) * Id + Efd) / self.Td0p,
                (-Ed + (self.Xq - self.Xqp) * Iq) / self.Tq0p,
                (-Efd + self.KA * (self.Vref - v[self.ksg])) / self.TA,
                (-Psv + self.Pref - (w - 1.0) / self.R) / self.Tg,
                (-Pm + Psv) / self.Tt]
        for t, r in enumerate(rows):
            out[o + t] = r
        tp, xp, xid, xiq, i_d, i_q, vdc, xdc = self.cv_states(x)
        phi = th[self.kcv] - tp
        vd = v[self.kcv] * np.cos(phi)
        vq = v[self.kcv] * np.sin(phi)
        idr = self.Kpdc * (vdc - self.Vdc0) + self.Kidc * xdc
        o = self.off[self.icv]
        rows = [self.ws * (self.Kpp * vq + self.Kip * xp),
                vq,
                idr - i_d,
                self.iq_ref - i_q,
                self.ws / self.Lf * (self.Kpc * (idr - i_d) + self.Kic * xid - self.Rf * i_d),
                self.ws / self.Lf * (self.Kpc * (self.iq_ref - i_q) + self.Kic * xiq
                                     - self.Rf * i_q),
                (self.Pdc - (vd * i_d + vq * i_q)) / (self.Cdc * vdc),
                vdc - self.Vdc0]
        for t, r in enumerate(rows):
            out[o + t] = r
        return out

    def g(self, x, y):
        Id, Iq, th, v = self.split(y)
        d, w, Eq, Ed = self.sg_states(x)[:4]
        a = d - th[self.ksg]
        vk = v[self.ksg]
        gd = Ed - vk * np.sin(a) - self.Rs * Id + self.Xqp * Iq
        gq = Eq - vk * np.cos(a) - self.Rs * Iq - self.Xdp * Id
        V = v * np.exp(1j * th)
        Snet = V * np.conj(self.sub.Y @ V)
        Pg = np.zeros(self.nb)
        Qg = np.zeros(self.nb)
        np.add.at(Pg, self.ksg, Id * vk * np.sin(a) + Iq * vk * np.cos(a))
        np.add.at(Qg, self.ksg, Id * vk * np.cos(a) - Iq * vk * np.sin(a))
        tp, _, _, _, i_d, i_q = self.cv_states(x)[:6]
        phi = th[self.kcv] - tp
        vc = v[self.kcv]
        np.add.at(Pg, self.kcv, vc * (i_d * np.cos(phi) + i_q * np.sin(phi)))
        np.add.at(Qg, self.kcv, vc * (i_d * np.sin(phi) - i_q * np.cos(phi)))
        r2 = (v / self.V0) ** 2
        gP = Pg - self.P0 * r2 - Snet.real
        gQ = Qg - self.Q0 * r2 - Snet.imag
        return np.concatenate([gd, gq, gP, gQ])

    # --- analytic Jacobians at (x0, y0) ----------------------------------
    def jacobians(self):
        nsg, nb = self.nsg, self.nb
        x, y = self.x0, self.y0
        Id, Iq, th, v = self.split(y)
        nx = self.nx
        ny = 2 * nsg + 2 * nb
        fx = np.zeros((nx, nx))
        fy = np.zeros((nx, ny))
        gx = np.zeros((ny, nx))
        gy = np.zeros((ny, ny))
        cth0, cv0 = 2 * nsg, 2 * nsg + nb          # theta, V columns
        # ---------------- synchronous machines
        d, w, Eq, Ed = self.sg_states(x)[:4]
        k = self.ksg
        a = d - th[k]
        vk = v[k]
        s, c = np.sin(a), np.cos(a)
        i = np.arange(nsg)
        r = self.off[self.isg]
        H2 = 2.0 * self.H
        fx[r, r + 1] = self.ws
        fx[r + 1, r + 1] = -self.D / H2
        fx[r + 1, r + 2] = -Iq / H2
        fx[r + 1, r + 3] = -Id / H2
        fx[r + 1, r + 6] = 1.0 / H2
        fx[r + 2, r + 2] = -1.0 / self.Td0p
        fx[r + 2, r + 4] = 1.0 / self.Td0p
        fx[r + 3, r + 3] = -1.0 / self.Tq0p
        fx[r + 4, r + 4] = -1.0 / self.TA
        fx[r + 5, r + 1] = -1.0 / (self.R * self.Tg)
        fx[r + 5, r + 5] = -1.0 / self.Tg
        fx[r + 6, r + 5] = 1.0 / self.Tt
        fx[r + 6, r + 6] = -1.0 / self.Tt
        cId, cIq = i, nsg + i
        cth, cv = cth0 + k, cv0 + k
        fy[r + 1, cId] = -(Ed + (self.Xqp - self.Xdp) * Iq) / H2
        fy[r + 1, cIq] = -(Eq + (self.Xqp - self.Xdp) * Id) / H2
        fy[r + 2, cId] = -(self.Xd - self.Xdp) / self.Td0p
        fy[r + 3, cIq] = (self.Xq - self.Xqp) / self.Tq0p
        fy[r + 4, cv] = -self.KA / self.TA
        # stator rows
        gx[i, r] = -vk * c
        gx[i, r + 3] = 1.0
        gx[nsg + i, r] = vk * s
        gx[nsg + i, r + 2] = 1.0
        # network rows: machine injection
        rP, rQ = cth0 + k, cv0 + k
        dPdd = Id * vk * c - Iq * vk * s
        dQdd = -Id * vk * s - Iq * vk * c
        np.add.at(gx, (rP, r), dPdd)
        np.add.at(gx, (rQ, r), dQdd)
        gy[i, cId] = -self.Rs
        gy[i, cIq] = self.Xqp
        gy[i, cth] = vk * c
        gy[i, cv] = -s
        gy[nsg + i, cId] = -self.Xdp
        gy[nsg + i, cIq] = -self.Rs
        gy[nsg + i, cth] = -vk * s
        gy[nsg + i, cv] = -c
        np.add.at(gy, (rP, cId), vk * s)
        np.add.at(gy, (rP, cIq), vk * c)
        np.add.at(gy, (rP, cth), -dPdd)
        np.add.at(gy, (rP, cv), Id * s + Iq * c)
        np.add.at(gy, (rQ, cId), vk * c)
        np.add.at(gy, (rQ, cIq), -vk * s)
        np.add.at(gy, (rQ, cth), -dQdd)
        np.add.at(gy, (rQ, cv), Id * c - Iq * s)
        # ---------------- converters
        tp, xp, xid, xiq, i_d, i_q, vdc, xdc = self.cv_states(x)
        k = self.kcv
        r = self.off[self.icv]
        vc = v[k]
        phi = th[k] - tp
        cp, sp = np.cos(phi), np.sin(phi)
        vd, vq = vc * cp, vc * sp
        ws = self.ws
        g_ = ws / self.Lf
        cdv = self.Cdc * vdc
        # v_d = V cos(phi), v_q = V sin(phi), phi = theta - theta_p
        dvd = dict(tp=vq, th=-vq, V=cp)
        dvq = dict(tp=-vd, th=vd, V=sp)
        # theta_p, x_pll
        fx[r, r] = ws * self.Kpp * dvq["tp"]
        fx[r, r + 1] = ws * self.Kip
        fy[r, cth0 + k] = ws * self.Kpp * dvq["th"]
        fy[r, cv0 + k] = ws * self.Kpp * dvq["V"]
        fx[r + 1, r] = dvq["tp"]
        fy[r + 1, cth0 + k] = dvq["th"]
        fy[r + 1, cv0 + k] = dvq["V"]
        # current-loop integrators
        fx[r + 2, r + 4] = -1.0
        fx[r + 2, r + 6] = self.Kpdc
        fx[r + 2, r + 7] = self.Kidc
        fx[r + 3, r + 5] = -1.0
        # filter currents
        fx[r + 4, r + 4] = -g_ * (self.Kpc + self.Rf)
        fx[r + 4, r + 2] = g_ * self.Kic
        fx[r + 4, r + 6] = g_ * self.Kpc * self.Kpdc
        fx[r + 4, r + 7] = g_ * self.Kpc * self.Kidc
        fx[r + 5, r + 5] = -g_ * (self.Kpc + self.Rf)
        fx[r + 5, r + 3] = g_ * self.Kic
        # DC link: f = (Pdc - Pac) / (Cdc v_dc), Pac = v_d i_d + v_q i_q
        num = self.Pdc - (vd * i_d + vq * i_q)
        fx[r + 6, r + 6] = -num / (cdv * vdc)
        fx[r + 6, r] = -(i_d * dvd["tp"] + i_q * dvq["tp"]) / cdv
        fx[r + 6, r + 4] = -vd / cdv
        fx[r + 6, r + 5] = -vq / cdv
        fy[r + 6, cth0 + k] = -(i_d * dvd["th"] + i_q * dvq["th"]) / cdv
        fy[r + 6, cv0 + k] = -(i_d * dvd["V"] + i_q * dvq["V"]) / cdv
        fx[r + 7, r + 6] = 1.0
        # network rows: converter injection
        rP, rQ = cth0 + k, cv0 + k
        Pc = vc * (i_d * cp + i_q * sp)
        Qc = vc * (i_d * sp - i_q * cp)
        dPdphi = vc * (-i_d * sp + i_q * cp)
        dQdphi = vc * (i_d * cp + i_q * sp)
        np.add.at(gx, (rP, r), -dPdphi)
        np.add.at(gx, (rQ, r), -dQdphi)
        np.add.at(gx, (rP, r + 4), vc * cp)
        np.add.at(gx, (rP, r + 5), vc * sp)
        np.add.at(gx, (rQ, r + 4), vc * sp)
        np.add.at(gx, (rQ, r + 5), -vc * cp)
        np.add.at(gy, (rP, cth0 + k), dPdphi)
        np.add.at(gy, (rQ, cth0 + k), dQdphi)
        np.add.at(gy, (rP, cv0 + k), Pc / vc)
        np.add.at(gy, (rQ, cv0 + k), Qc / vc)
        # ---------------- loads and network
        b = np.arange(nb)
        gy[cth0 + b, cv0 + b] -= 2.0 * self.P0 * v / self.V0 ** 2
        gy[cv0 + b, cv0 + b] -= 2.0 * self.Q0 * v / self.V0 ** 2
        V = v * np.exp(1j * th)
        _, dth, dvm = complex_power_jac(self.sub.Y, b, V)
        gy[cth0:cth0 + nb, cth0:cth0 + nb] -= dth.real
        gy[cth0:cth0 + nb, cv0:] -= dvm.real
        gy[cv0:, cth0:cth0 + nb] -= dth.imag
        gy[cv0:, cv0:] -= dvm.imag
        return fx, fy, gx, gy

    def state_matrix_full(self):
        fx, fy, gx, gy = self.jacobians()
        return fx - fy @ np.linalg.solve(gy, gx)

    def state_matrix(self):
        """Relative-angle state matrix (n = 7 n_SG + 8 n_GFL - 1)."""
        return reduce_relative_angles(self.state_matrix_full(), self.off)


def reduce_relative_angles(A, offsets):
    """Angles relative to the first device: every other device's angle row
    (local state 0 of both kinds) minus the first one's, then the first
    angle's row and column removed.  offsets: first state of every device
    (an int n_devices means synchronous machines only, NS_SG states each)."""
    if np.isscalar(offsets):
        offsets = NS_SG * np.arange(int(offsets))
    A = A.copy()
    ref = int(offsets[0])
    for o in offsets[1:]:
        A[int(o)] -= A[ref]
    keep = np.array([j for j in range(A.shape[0]) if j != ref])
    return A[np.ix_(keep, keep)]
