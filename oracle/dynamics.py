"""Linearised state matrix at the OPF operating point (Section II.B.2).

The paper builds the full dynamic model at the OPF point, linearises it and
inspects the eigenvalues of the state matrix; it leaves the device models to
its simulation tool.  The oracle uses the standard phasor models of Sauer and
Pai (Power System Dynamics and Stability):

Synchronous generator, two-axis model, states
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
network (algebraic, per island bus): generator injections
  P = Id V sin(delta-theta) + Iq V cos(delta-theta),
  Q = Id V cos(delta-theta) - Iq V sin(delta-theta)
minus constant-impedance loads P0 (V/V0)^2, Q0 (V/V0)^2 (V0 the OPF voltage)
minus the network injection V conj(Y V).

Algebraic variables y = [Id, Iq, theta, V].  Linearisation:
  A_full = f_x - f_y g_y^{-1} g_x.
The absolute rotor angles leave a structural zero eigenvalue (a uniform shift
of every angle is an equilibrium).  It is removed by taking angles relative to
the first machine: every other delta row minus that machine's delta row, then
its delta row and column deleted.
"""
from __future__ import annotations

import numpy as np

from .opf import complex_power_jac

NS_SG = 7       # states per synchronous generator


class DynModel:
    def __init__(self, net, sub, vm, va, pg, qg):
        if np.any(net["gen_kind"][sub.gen] != 0):
            raise NotImplementedError("only synchronous generators")
        self.sub = sub
        self.ng = ng = len(sub.gen)
        self.nb = nb = sub.nb
        self.ws = 2.0 * np.pi * float(net["f_hz"])
        p = net["dyn"][sub.gen]
        (self.H, self.D, self.Xd, self.Xq, self.Xdp, self.Xqp, self.Td0p,
         self.Tq0p, self.Rs, self.KA, self.TA, self.R, self.Tg,
         self.Tt) = p.T
        self.k = sub.gbus
        self.P0 = sub.pd.copy()
        self.Q0 = sub.qd.copy()
        self.V0 = vm.copy()
        # --- equilibrium from the operating point -------------------------
        V = vm * np.exp(1j * va)
        Vg = V[self.k]
        I = np.conj((pg + 1j * qg) / Vg)
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
        self.Vref = vm[self.k] + np.where(self.KA != 0.0, Efd / safe, 0.0)
        Pm = Edp * Id + Eqp * Iq + (self.Xqp - self.Xdp) * Id * Iq
        self.Pref = Pm.copy()
        x = np.stack([delta, np.ones(ng), Eqp, Edp, Efd, Pm, Pm], axis=1)
        self.x0 = x.reshape(-1)
        self.y0 = np.concatenate([Id, Iq, va, vm])

    # --- residuals --------------------------------------------------------
    def split(self, x, y):
        ng, nb = self.ng, self.nb
        X = x.reshape(ng, NS_SG)
        Id, Iq = y[:ng], y[ng:2 * ng]
        th, v = y[2 * ng:2 * ng + nb], y[2 * ng + nb:]
        return X, Id, Iq, th, v

    def f(self, x, y):
        X, Id, Iq, th, v = self.split(x, y)
        d, w, Eq, Ed, Efd, Psv, Pm = X.T
        Pe = Ed * Id + Eq * Iq + (self.Xqp - self.Xdp) * Id * Iq
        out = np.stack([
            self.ws * (w - 1.0),
            (Pm - Pe - self.D * (w - 1.0)) / (2.0 * self.H),
            (-Eq - (self.Xd - self.Xdp) * Id + Efd) / self.Td0p,
            (-Ed + (self.Xq - self.Xqp) * Iq) / self.Tq0p,
            (-Efd + self.KA * (self.Vref - v[self.k])) / self.TA,
            (-Psv + self.Pref - (w - 1.0) / self.R) / self.Tg,
            (-Pm + Psv) / self.Tt], axis=1)
        return out.reshape(-1)

    def g(self, x, y):
        X, Id, Iq, th, v = self.split(x, y)
        d = X[:, 0]
        Ed, Eq = X[:, 3], X[:, 2]
        a = d - th[self.k]
        vk = v[self.k]
        gd = Ed - vk * np.sin(a) - self.Rs * Id + self.Xqp * Iq
        gq = Eq - vk * np.cos(a) - self.Rs * Iq - self.Xdp * Id
        V = v * np.exp(1j * th)
        Snet = V * np.conj(self.sub.Y @ V)
        Pg = np.zeros(self.nb)
        Qg = np.zeros(self.nb)
        np.add.at(Pg, self.k, Id * vk * np.sin(a) + Iq * vk * np.cos(a))
        np.add.at(Qg, self.k, Id * vk * np.cos(a) - Iq * vk * np.sin(a))
        r2 = (v / self.V0) ** 2
        gP = Pg - self.P0 * r2 - Snet.real
        gQ = Qg - self.Q0 * r2 - Snet.imag
        return np.concatenate([gd, gq, gP, gQ])

    # --- analytic Jacobians ----------------------------------------------
    def jacobians(self):
        ng, nb = self.ng, self.nb
        x, y = self.x0, self.y0
        X, Id, Iq, th, v = self.split(x, y)
        d, w, Eq, Ed = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
        k = self.k
        a = d - th[k]
        vk = v[k]
        s, c = np.sin(a), np.cos(a)
        nx = NS_SG * ng
        ny = 2 * ng + 2 * nb
        fx = np.zeros((nx, nx))
        fy = np.zeros((nx, ny))
        gx = np.zeros((ny, nx))
        gy = np.zeros((ny, ny))
        i = np.arange(ng)
        r = NS_SG * i
        H2 = 2.0 * self.H
        # f_x
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
        # f_y
        cId, cIq = i, ng + i
        cth, cv = 2 * ng + k, 2 * ng + nb + k
        fy[r + 1, cId] = -(Ed + (self.Xqp - self.Xdp) * Iq) / H2
        fy[r + 1, cIq] = -(Eq + (self.Xqp - self.Xdp) * Id) / H2
        fy[r + 2, cId] = -(self.Xd - self.Xdp) / self.Td0p
        fy[r + 3, cIq] = (self.Xq - self.Xqp) / self.Tq0p
        fy[r + 4, cv] = -self.KA / self.TA
        # g_x: stator rows
        gx[i, r] = -vk * c
        gx[i, r + 3] = 1.0
        gx[ng + i, r] = vk * s
        gx[ng + i, r + 2] = 1.0
        # g_x: network rows (generator injection depends on delta)
        rP, rQ = 2 * ng + k, 2 * ng + nb + k
        dPdd = Id * vk * c - Iq * vk * s
        dQdd = -Id * vk * s - Iq * vk * c
        np.add.at(gx, (rP, r), dPdd)
        np.add.at(gx, (rQ, r), dQdd)
        # g_y: stator rows
        gy[i, cId] = -self.Rs
        gy[i, cIq] = self.Xqp
        gy[i, cth] = vk * c
        gy[i, cv] = -s
        gy[ng + i, cId] = -self.Xdp
        gy[ng + i, cIq] = -self.Rs
        gy[ng + i, cth] = -vk * s
        gy[ng + i, cv] = -c
        # g_y: network rows, generator part
        np.add.at(gy, (rP, cId), vk * s)
        np.add.at(gy, (rP, cIq), vk * c)
        np.add.at(gy, (rP, cth), -dPdd)
        np.add.at(gy, (rP, cv), Id * s + Iq * c)
        np.add.at(gy, (rQ, cId), vk * c)
        np.add.at(gy, (rQ, cIq), -vk * s)
        np.add.at(gy, (rQ, cth), -dQdd)
        np.add.at(gy, (rQ, cv), Id * c - Iq * s)
        # g_y: loads and network
        b = np.arange(nb)
        gy[2 * ng + b, 2 * ng + nb + b] -= 2.0 * self.P0 * v / self.V0 ** 2
        gy[2 * ng + nb + b, 2 * ng + nb + b] -= 2.0 * self.Q0 * v / self.V0 ** 2
        V = v * np.exp(1j * th)
        _, dth, dvm = complex_power_jac(self.sub.Y, b, V)
        gy[2 * ng:2 * ng + nb, 2 * ng:2 * ng + nb] -= dth.real
        gy[2 * ng:2 * ng + nb, 2 * ng + nb:] -= dvm.real
        gy[2 * ng + nb:, 2 * ng:2 * ng + nb] -= dth.imag
        gy[2 * ng + nb:, 2 * ng + nb:] -= dvm.imag
        return fx, fy, gx, gy

    def state_matrix_full(self):
        fx, fy, gx, gy = self.jacobians()
        return fx - fy @ np.linalg.solve(gy, gx)

    def state_matrix(self):
        """Relative-angle state matrix (n = 7 ng - 1)."""
        A = self.state_matrix_full()
        return reduce_relative_angles(A, self.ng)


def reduce_relative_angles(A, ng):
    """Angles relative to machine 0: delta_i rows minus delta_0's row, then
    delta_0's row and column removed."""
    A = A.copy()
    d0 = 0
    for i in range(1, ng):
        A[NS_SG * i] -= A[d0]
    keep = np.array([j for j in range(A.shape[0]) if j != d0])
    return A[np.ix_(keep, keep)]
