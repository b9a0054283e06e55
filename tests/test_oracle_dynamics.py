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
    assert len(lr) == len(lf) - 1 == 7 * dm.ng - 1
    assert np.min(np.abs(lr)) > 1e-6
    d = np.array([np.min(np.abs(others - z)) for z in lr])
    assert np.max(d) < 1e-8 * max(1.0, np.abs(lr).max())
    # the null vector of the full matrix is the uniform angle shift
    _, _, vh = np.linalg.svd(Af)
    v = vh[-1] / np.max(np.abs(vh[-1]))
    shift = np.zeros(Af.shape[0])
    shift[::dynamics.NS_SG] = 1.0
    assert np.allclose(np.abs(v), shift, atol=1e-6)
