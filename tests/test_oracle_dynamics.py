"""Pins for the linearised state matrix (Section II.B.2).

* Two identical classical machines (transient saliency removed, fluxes
  frozen by huge open-circuit constants, no AVR gain, no governor droop)
  tied by a lossless line: the electromechanical pair is
  s = -D/(4H) +- j sqrt(ws Ks / H - (D/4H)^2), Ks = E1 E2 cos(d12) / Xt,
  with internal voltages E = V + j Xd' I from the textbook model.
* A single machine against an infinite bus (the other machine's inertia and
  damping scaled by 1e7): 2H s^2 + D s + ws Ks = 0.
* The equilibrium built from the OPF point satisfies f = 0 and g = 0.
* The analytic Jacobians match central differences of f and g.
* The full matrix has one eigenvalue at 0 (uniform angle shift) that the
  relative-angle reduction removes, leaving the rest unchanged.
"""
import numpy as np
import pytest

from inputs import netgen
from oracle import opf, dynamics, eigen
from nets import make_net, full_subsystem, base_dyn_row
import os

CASES = os.path.join(os.path.dirname(os.path.dirname(__file__)), "inputs", "cases")


def _classical_pair(H=4.0, D=3.0, xl=0.2, xdp=0.3):
    row = base_dyn_row(H=H, D=D, Xd=xdp, Xq=xdp, Xdp=xdp, Xqp=xdp,
                       Td0p=1e9, Tq0p=1e9, KA=0.0, R=1e12)
    gens = [dict(bus=0, pmin=-2.0, pmax=2.0, c2=0.01, c1=0.0, dyn=row),
            dict(bus=1, pmin=-0.5, pmax=2.0, c2=0.01, c1=50.0, dyn=row)]
    return make_net(2, [(0, 1, 0.0, xl, 0.0)], gens, [], vmin=0.95, vmax=1.05)


def test_two_machine_classical_closed_form():
    H, D, xl, xdp = 4.0, 3.0, 0.2, 0.3
    net = _classical_pair(H, D, xl, xdp)
    sub = full_subsystem(net)
    o = opf.solve_opf(net, sub)
    assert o.status == opf.CONVERGED
    assert o.pg[1] < -0.4                      # power flows from machine 0 to 1
    V = o.vm * np.exp(1j * o.va)
    I = np.conj((o.pg + 1j * o.qg) / V)
    E = V + 1j * xdp * I
    Ks = abs(E[0]) * abs(E[1]) * np.cos(np.angle(E[0]) - np.angle(E[1])) / (2 * xdp + xl)
    ws = 2 * np.pi * 60.0
    w = np.sqrt(ws * Ks / H - (D / (4 * H)) ** 2)
    s_expected = complex(-D / (4 * H), w)
    lam = eigen.eigvals(dynamics.DynModel(net, sub, o.vm, o.va, o.pg, o.qg).state_matrix())
    k = np.argmin(np.abs(lam - s_expected))
    assert abs(lam[k] - s_expected) < 1e-6 * abs(s_expected)
    # common-mode speed deviation decays at -D/(2H)
    assert np.min(np.abs(lam - (-D / (2 * H)))) < 1e-6


def test_single_machine_infinite_bus_closed_form():
    """Machine 1 with an inertia 1e7 times larger acts as an infinite bus:
    the electromechanical mode of machine 0 is the SMIB root of
    2H s^2 + D s + ws Ks = 0, s = -D/(4H) +- j sqrt(ws Ks / (2H) - (D/4H)^2)."""
    H, D, xl, xdp = 4.0, 3.0, 0.2, 0.3
    net = _classical_pair(H, D, xl, xdp)
    big = 1e7
    net["dyn"][1, netgen.DYN_COLS.index("H")] = H * big
    net["dyn"][1, netgen.DYN_COLS.index("D")] = D * big
    sub = full_subsystem(net)
    o = opf.solve_opf(net, sub)
    assert o.status == opf.CONVERGED
    V = o.vm * np.exp(1j * o.va)
    I = np.conj((o.pg + 1j * o.qg) / V)
    E = V + 1j * xdp * I
    Ks = abs(E[0]) * abs(E[1]) * np.cos(np.angle(E[0]) - np.angle(E[1])) / (2 * xdp + xl)
    ws = 2 * np.pi * 60.0
    w = np.sqrt(ws * Ks / (2 * H) - (D / (4 * H)) ** 2)
    s_expected = complex(-D / (4 * H), w)
    lam = eigen.eigvals(dynamics.DynModel(net, sub, o.vm, o.va, o.pg, o.qg).state_matrix())
    k = np.argmin(np.abs(lam - s_expected))
    assert abs(lam[k] - s_expected) < 1e-5 * abs(s_expected)


@pytest.fixture(scope="module")
def c1_base():
    net = netgen.load_case(os.path.join(CASES, "c1_30.npz"))
    sub = full_subsystem(net)
    o = opf.solve_opf(net, sub)
    assert o.status == opf.CONVERGED
    return net, sub, o, dynamics.DynModel(net, sub, o.vm, o.va, o.pg, o.qg)


def test_equilibrium(c1_base):
    net, sub, o, dm = c1_base
    assert np.max(np.abs(dm.f(dm.x0, dm.y0))) < 1e-10
    # network rows hold to the OPF's balance tolerance
    assert np.max(np.abs(dm.g(dm.x0, dm.y0))) < 1e-8


def test_jacobians_central_differences(c1_base):
    net, sub, o, dm = c1_base
    fx, fy, gx, gy = dm.jacobians()
    eps = 1e-6
    for J, fun, which in [(fx, dm.f, "x"), (fy, dm.f, "y"), (gx, dm.g, "x"), (gy, dm.g, "y")]:
        z0 = dm.x0 if which == "x" else dm.y0
        for k in range(len(z0)):
            e = np.zeros(len(z0))
            e[k] = eps
            if which == "x":
                d = (fun(z0 + e, dm.y0) - fun(z0 - e, dm.y0)) / (2 * eps)
            else:
                d = (fun(dm.x0, z0 + e) - fun(dm.x0, z0 - e)) / (2 * eps)
            assert np.allclose(d, J[:, k], atol=2e-6, rtol=1e-6)


def test_structural_zero_removed(c1_base):
    net, sub, o, dm = c1_base
    Af = dm.state_matrix_full()
    lf = np.linalg.eigvals(Af)
    k = np.argmin(np.abs(lf))
    assert abs(lf[k]) < 1e-9 * np.linalg.norm(Af)
    others = np.sort_complex(np.delete(lf, k))
    lr = np.sort_complex(np.linalg.eigvals(dm.state_matrix()))
    assert len(lr) == len(lf) - 1 == 7 * dm.nsg - 1
    assert np.min(np.abs(lr)) > 1e-6
    d = np.array([np.min(np.abs(others - z)) for z in lr])
    assert np.max(d) < 1e-8 * max(1.0, np.abs(lr).max())
    # the null vector of the full matrix is the uniform angle shift
    _, _, vh = np.linalg.svd(Af)
    v = vh[-1] / np.max(np.abs(vh[-1]))
    shift = np.zeros(Af.shape[0])
    shift[::dynamics.NS_SG] = 1.0
    assert np.allclose(np.abs(v), shift, atol=1e-6)


# --- single machine against an infinite bus, every model row live -----------
#
# Bus 1 holds the machine under test (two-axis with transient saliency, AVR,
# governor and turbine, no time constant frozen); bus 0 holds machine 0 with
# Xd' = Xq' = Xp0, which is a constant EMF E_inf behind Xp0 while its own
# states are held (A's entries are partial derivatives).  With a lossless line
# x and no loads, machine 1 sees E_inf behind Xe = x + Xp0, and in its own dq
# frame the network reduces to
#     Vd = E_b sin d - Xe Iq,   Vq = E_b cos d + Xe Id     (d = delta - arg E_inf)
# which with the stator (Rs = 0) Vd = Ed' + Xq' Iq, Vq = Eq' - Xd' Id gives
#     Id = (Eq' - E_b cos d) / (Xe + Xd'),   Iq = (E_b sin d - Ed') / (Xe + Xq').
# Linearising Pe = Ed' Id + Eq' Iq + (Xq' - Xd') Id Iq and |V| gives the
# Heffron-Phillips constants (deMello and Concordia 1969; Kundur, Power
# System Stability and Control, Section 12.3) extended by the q-axis EMF:
#     dPe = K1 dd + K2 dEq' + K2d dEd',   dV = K5 dd + K6 dEq' + K6d dEd',
#     1/K3 = (Xd + Xe)/(Xd' + Xe),  K4 = (Xd - Xd') E_b sin d / (Xd' + Xe),
#     1/K3d = (Xq + Xe)/(Xq' + Xe), K4d = (Xq - Xq') E_b cos d / (Xq' + Xe).

def _smib_case(V0=1.0, V1=1.03, th1=0.25, x=0.3, Xp0=0.05):
    row0 = base_dyn_row(Xd=0.9, Xq=0.8, Xdp=Xp0, Xqp=Xp0)
    row1 = base_dyn_row()            # H 4, D 2, Xd 1.5, Xq 1.4, Xd' 0.3, Xq' 0.5, ...
    gens = [dict(bus=0, pmin=-5, pmax=5, qmin=-5, qmax=5, dyn=row0),
            dict(bus=1, pmin=-5, pmax=5, qmin=-5, qmax=5, dyn=row1)]
    net = make_net(2, [(0, 1, 0.0, x, 0.0)], gens, [])
    Vb = np.array([V0 + 0j, V1 * np.exp(1j * th1)])
    I1 = (Vb[1] - Vb[0]) / (1j * x)             # injected by machine 1
    S = Vb * np.conj(np.array([-I1, I1]))
    return net, Vb, I1, S, x + Xp0, dict(zip(netgen.DYN_COLS, row1))


def _smib_closed_form(Vb, I1, Xe, p, ws):
    Xd, Xq, Xdp, Xqp = p["Xd"], p["Xq"], p["Xdp"], p["Xqp"]
    H, D, KA, TA, R, Tg, Tt = p["H"], p["D"], p["KA"], p["TA"], p["R"], p["Tg"], p["Tt"]
    Td0p, Tq0p = p["Td0p"], p["Tq0p"]
    Einf = Vb[1] - 1j * Xe * I1
    delta = np.angle(Vb[1] + 1j * Xq * I1)
    rot = np.exp(-1j * (delta - np.pi / 2))
    Idq, Vdq = I1 * rot, Vb[1] * rot
    Id, Iq, Vd, Vq = Idq.real, Idq.imag, Vdq.real, Vdq.imag
    Edp, Eqp = Vd - Xqp * Iq, Vq + Xdp * Id
    Eb, d = abs(Einf), delta - np.angle(Einf)
    # the reduced network reproduces the operating point
    assert abs(Id - (Eqp - Eb * np.cos(d)) / (Xe + Xdp)) < 1e-12
    assert abs(Iq - (Eb * np.sin(d) - Edp) / (Xe + Xqp)) < 1e-12
    dId_dd, dIq_dd = Eb * np.sin(d) / (Xe + Xdp), Eb * np.cos(d) / (Xe + Xqp)
    ad, aq = Edp + (Xqp - Xdp) * Iq, Eqp + (Xqp - Xdp) * Id
    K1 = ad * dId_dd + aq * dIq_dd
    K2 = Iq + ad / (Xe + Xdp)
    K2d = Id - aq / (Xe + Xqp)
    K3 = (Xdp + Xe) / (Xd + Xe)
    K4 = (Xd - Xdp) * Eb * np.sin(d) / (Xdp + Xe)
    K3d = (Xqp + Xe) / (Xq + Xe)
    K4d = (Xq - Xqp) * Eb * np.cos(d) / (Xqp + Xe)
    V = abs(Vb[1])
    K5 = (Vd * Xqp * dIq_dd - Vq * Xdp * dId_dd) / V
    K6 = Vq / V * Xe / (Xe + Xdp)
    K6d = Vd / V * Xe / (Xe + Xqp)
    H2 = 2 * H
    # states: delta, omega, Eq', Ed', Efd, Psv, Pm
    return np.array([
        [0, ws, 0, 0, 0, 0, 0],
        [-K1 / H2, -D / H2, -K2 / H2, -K2d / H2, 0, 0, 1 / H2],
        [-K4 / Td0p, 0, -1 / (K3 * Td0p), 0, 1 / Td0p, 0, 0],
        [K4d / Tq0p, 0, 0, -1 / (K3d * Tq0p), 0, 0, 0],
        [-KA * K5 / TA, 0, -KA * K6 / TA, -KA * K6d / TA, -1 / TA, 0, 0],
        [0, -1 / (R * Tg), 0, 0, 0, -1 / Tg, 0],
        [0, 0, 0, 0, 0, 1 / Tt, -1 / Tt]])


@pytest.mark.parametrize("V1,th1,x", [(1.03, 0.25, 0.3), (0.97, -0.4, 0.2), (1.05, 0.6, 0.45)])
def test_smib_two_axis_avr_governor_heffron_phillips(V1, th1, x):
    """Machine 1's 7 x 7 block of the oracle's state matrix, entry by entry,
    against the Heffron-Phillips form above (rotor angle, speed, both
    transient EMFs, exciter, governor and turbine rows)."""
    net, Vb, I1, S, Xe, p = _smib_case(V1=V1, th1=th1, x=x)
    sub = full_subsystem(net)
    dm = dynamics.DynModel(net, sub, np.abs(Vb), np.angle(Vb), S.real, S.imag)
    # the equilibrium is one (f = 0, g = 0 at the given point)
    assert np.max(np.abs(dm.f(dm.x0, dm.y0))) < 1e-12
    assert np.max(np.abs(dm.g(dm.x0, dm.y0))) < 1e-12
    A = dm.state_matrix()
    assert A.shape == (13, 13)
    blk = A[6:13, 6:13]               # [delta1 - delta0, omega1, Eq1', Ed1', Efd1, Psv1, Pm1]
    ref = _smib_closed_form(Vb, I1, Xe, p, dm.ws)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(blk - ref)) < 1e-11 * scale, np.abs(blk - ref).max()
    # eigenvalues of the block are the roots of its characteristic polynomial
    lam_ref = np.roots(np.poly(ref))
    from helpers import match_eigs
    assert match_eigs(eigen.eigvals(blk), lam_ref) < 1e-8


# --- grid-following converters -------------------------------------------------
#
# A converter at bus 1 fed against an infinite bus (machine 0 with Xd' = Xq',
# a constant EMF E_inf behind Xp0 while its states are held) through a
# lossless line x.  With Xe = x + Xp0 and the injected current
# (i_d + j i_q) e^{j theta_p}, the terminal voltage in the PLL frame is
#     v_d + j v_q = E e^{-j t} + j Xe (i_d + j i_q),   t = theta_p - arg E_inf
# so v_d = E cos t - Xe i_q, v_q = -E sin t + Xe i_d (the PLL sees the
# converter's own current through the grid impedance).  Differentiating the
# converter's eight equations with that elimination gives its 8 x 8 block in
# closed form (below), which the oracle's network-level linearisation must
# reproduce entry by entry.

def gfl_row(**kw):
    d = dict(Kpp=0.1, Kip=2.0, Kpc=0.45, Kic=10.0, Lf=0.15, Rf=0.01, Cdc=0.08, Kpdc=2.0,
             Kidc=20.0, Vdc0=1.0)
    d.update(kw)
    row = [d[k] for k in dynamics.GFL_COLS]
    return row + [1.0] * (netgen.N_DYN - len(row))


def _gfl_smib(V0=1.0, V1=1.02, th1=0.2, x=0.25, Xp0=0.05, **kw):
    row0 = base_dyn_row(Xd=0.9, Xq=0.8, Xdp=Xp0, Xqp=Xp0)
    gens = [dict(bus=0, pmin=-5, pmax=5, qmin=-5, qmax=5, dyn=row0),
            dict(bus=1, pmin=-5, pmax=5, qmin=-5, qmax=5, dyn=gfl_row(**kw))]
    net = make_net(2, [(0, 1, 0.0, x, 0.0)], gens, [])
    net["gen_kind"] = np.array([0, 1], np.int32)
    Vb = np.array([V0 + 0j, V1 * np.exp(1j * th1)])
    I1 = (Vb[1] - Vb[0]) / (1j * x)
    S = Vb * np.conj(np.array([-I1, I1]))
    p = dict(zip(dynamics.GFL_COLS, gfl_row(**kw)))
    return net, Vb, I1, S, x + Xp0, p


def _gfl_closed_form(Vb, I1, Xe, p, ws):
    Kpp, Kip, Kpc, Kic, Lf, Rf = p["Kpp"], p["Kip"], p["Kpc"], p["Kic"], p["Lf"], p["Rf"]
    Cdc, Kpdc, Kidc, Vdc0 = p["Cdc"], p["Kpdc"], p["Kidc"], p["Vdc0"]
    Einf = Vb[1] - 1j * Xe * I1
    tp = np.angle(Vb[1])                       # PLL locked to the terminal voltage
    idq = I1 * np.exp(-1j * tp)
    i_d, i_q = idq.real, idq.imag
    E, t = abs(Einf), tp - np.angle(Einf)
    vd, vq = E * np.cos(t) - Xe * i_q, -E * np.sin(t) + Xe * i_d
    assert abs(vq) < 1e-12 and abs(vd - abs(Vb[1])) < 1e-12
    Ec = E * np.cos(t)
    g = ws / Lf
    CV = Cdc * Vdc0
    A = np.zeros((8, 8))
    # states: theta_p, x_pll, x_id, x_iq, i_d, i_q, v_dc, x_dc
    A[0, [0, 1, 4]] = [-ws * Kpp * Ec, ws * Kip, ws * Kpp * Xe]
    A[1, [0, 4]] = [-Ec, Xe]
    A[2, [4, 6, 7]] = [-1.0, Kpdc, Kidc]
    A[3, 5] = -1.0
    A[4, [4, 2, 6, 7]] = [-g * (Kpc + Rf), g * Kic, g * Kpc * Kpdc, g * Kpc * Kidc]
    A[5, [5, 3]] = [-g * (Kpc + Rf), g * Kic]
    # dv_d/dtheta_p = -E sin t = -Xe i_d (v_q = 0), dv_q/dtheta_p = -E cos t
    A[6, [0, 4, 5]] = [(Xe * i_d * i_d + i_q * Ec) / CV, -(vd + Xe * i_q) / CV,
                       Xe * i_d / CV]
    A[7, 6] = 1.0
    return A


@pytest.mark.parametrize("V1,th1,x,kw", [(1.02, 0.2, 0.25, {}),
                                         (0.98, -0.3, 0.4, dict(Kpp=0.06, Kic=6.0)),
                                         (1.05, 0.5, 0.15, dict(Cdc=0.05, Kidc=12.0, Rf=0.02))])
def test_gfl_against_infinite_bus_closed_form(V1, th1, x, kw):
    net, Vb, I1, S, Xe, p = _gfl_smib(V1=V1, th1=th1, x=x, **kw)
    sub = full_subsystem(net)
    dm = dynamics.DynModel(net, sub, np.abs(Vb), np.angle(Vb), S.real, S.imag)
    assert np.max(np.abs(dm.f(dm.x0, dm.y0))) < 1e-12
    assert np.max(np.abs(dm.g(dm.x0, dm.y0))) < 1e-12
    A = dm.state_matrix()
    assert A.shape == (6 + 8, 6 + 8)
    blk = A[6:, 6:]
    ref = _gfl_closed_form(Vb, I1, Xe, p, dm.ws)
    assert np.max(np.abs(blk - ref)) < 1e-11 * np.max(np.abs(ref)), np.abs(blk - ref).max()


def test_pll_pair_on_a_stiff_bus():
    """With the grid impedance tending to zero the PLL decouples: its pair
    solves s^2 + ws Kpp V s + ws Kip V = 0."""
    net, Vb, I1, S, Xe, p = _gfl_smib(V1=1.0, th1=1e-4, x=1e-5, Xp0=1e-6)
    sub = full_subsystem(net)
    dm = dynamics.DynModel(net, sub, np.abs(Vb), np.angle(Vb), S.real, S.imag)
    blk = dm.state_matrix()[6:, 6:]
    ws, V = dm.ws, abs(Vb[1])
    roots = np.roots([1.0, ws * p["Kpp"] * V, ws * p["Kip"] * V])
    lam = eigen.eigvals(blk[:2, :2])
    from helpers import match_eigs
    assert match_eigs(roots, lam) < 1e-6


@pytest.fixture(scope="module")
def c1_mixed():
    """The 30-bus case with its generators 1 and 3 turned into converters."""
    net = netgen.load_case(os.path.join(CASES, "c1_30.npz"))
    net = dict(net)
    net["gen_kind"] = net["gen_kind"].copy()
    net["dyn"] = net["dyn"].copy()
    for g in (1, 3):
        net["gen_kind"][g] = 1
        net["dyn"][g] = gfl_row(Kpc=0.4 / net["pmax"][g], Kic=8.0 / net["pmax"][g],
                                Lf=0.12 / net["pmax"][g], Rf=0.01 / net["pmax"][g],
                                Cdc=0.07 * net["pmax"][g], Kpdc=2.0 * net["pmax"][g],
                                Kidc=15.0 * net["pmax"][g])
    sub = full_subsystem(net)
    o = opf.solve_opf(net, sub)
    assert o.status == opf.CONVERGED
    return net, sub, o, dynamics.DynModel(net, sub, o.vm, o.va, o.pg, o.qg)


def test_mixed_equilibrium_and_jacobians(c1_mixed):
    net, sub, o, dm = c1_mixed
    assert np.max(np.abs(dm.f(dm.x0, dm.y0))) < 1e-10
    assert np.max(np.abs(dm.g(dm.x0, dm.y0))) < 1e-8
    fx, fy, gx, gy = dm.jacobians()
    eps = 1e-6
    for J, fun, which in [(fx, dm.f, "x"), (fy, dm.f, "y"), (gx, dm.g, "x"), (gy, dm.g, "y")]:
        z0 = dm.x0 if which == "x" else dm.y0
        for k in range(len(z0)):
            e = np.zeros(len(z0))
            e[k] = eps
            if which == "x":
                d = (fun(z0 + e, dm.y0) - fun(z0 - e, dm.y0)) / (2 * eps)
            else:
                d = (fun(dm.x0, z0 + e) - fun(dm.x0, z0 - e)) / (2 * eps)
            assert np.allclose(d, J[:, k], atol=2e-6, rtol=1e-6), (which, k)


def test_mixed_structural_zero_removed(c1_mixed):
    """The uniform shift of every angle, rotor and PLL, is the null vector of
    the full matrix; the reduced one has 7 n_SG + 8 n_GFL - 1 states and the
    other eigenvalues unchanged."""
    net, sub, o, dm = c1_mixed
    Af = dm.state_matrix_full()
    lf = np.linalg.eigvals(Af)
    k = np.argmin(np.abs(lf))
    assert abs(lf[k]) < 1e-9 * np.linalg.norm(Af)
    _, _, vh = np.linalg.svd(Af)
    v = vh[-1] / np.max(np.abs(vh[-1]))
    shift = np.zeros(Af.shape[0])
    shift[dm.off] = 1.0
    assert np.allclose(np.abs(v), shift, atol=1e-6)
    lr = np.linalg.eigvals(dm.state_matrix())
    assert len(lr) == 7 * 4 + 8 * 2 - 1
    others = np.delete(lf, k)
    d = np.array([np.min(np.abs(others - z)) for z in lr])
    assert np.max(d) < 1e-8 * max(1.0, np.abs(lr).max())
