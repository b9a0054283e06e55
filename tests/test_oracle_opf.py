"""Pins for the oracle's AC OPF (Section II.B.1).

Closed forms: the two-bus radial feeder (high-voltage root of the receiving
voltage; optimum at the sending-end voltage cap since losses fall with
voltage) and lossless economic dispatch (equal incremental cost).  The
derivatives are checked against central differences of the constraint
functions, and every returned optimum is checked for its KKT certificate.
"""
import numpy as np
import pytest

from oracle import opf, network
from nets import make_net, full_subsystem


def _two_bus(P, Q, r, x, c2=0.05):
    return make_net(2, [(0, 1, r, x, 0.0)],
                    [dict(bus=0, pmax=10.0, qmin=-10.0, qmax=10.0, c2=c2)],
                    [(1, P, Q)], vmin=0.9, vmax=1.1)


@pytest.mark.parametrize("P,Q,r,x", [(0.8, 0.3, 0.02, 0.1), (1.2, 0.4, 0.03, 0.12),
                                     (0.3, 0.1, 0.01, 0.05)])
def test_two_bus_closed_form(P, Q, r, x):
    net = _two_bus(P, Q, r, x)
    o = opf.solve_opf(net, full_subsystem(net))
    assert o.status == opf.CONVERGED
    V1 = 1.1
    a = V1 ** 2 - 2 * (r * P + x * Q)
    v2sq = 0.5 * (a + np.sqrt(a * a - 4 * (r * r + x * x) * (P * P + Q * Q)))
    pg = P + r * (P * P + Q * Q) / v2sq
    assert abs(o.vm[0] - V1) < 1e-7
    assert abs(o.vm[1] - np.sqrt(v2sq)) < 1e-7
    assert abs(o.pg[0] - pg) < 1e-7
    assert abs(o.cost - 0.05 * (100 * pg) ** 2) < 1e-6 * o.cost


def _two_gen(c2a, c2b, pd, pmax_a=10.0):
    return make_net(2, [(0, 1, 0.0, 0.1, 0.0)],
                    [dict(bus=0, pmax=pmax_a, c2=c2a), dict(bus=1, pmax=10.0, c2=c2b)],
                    [(1, pd, 0.2)])


def test_lossless_economic_dispatch():
    c2a, c2b, pd = 0.02, 0.05, 1.4
    net = _two_gen(c2a, c2b, pd)
    o = opf.solve_opf(net, full_subsystem(net))
    assert o.status == opf.CONVERGED
    pa = pd * c2b / (c2a + c2b)
    assert abs(o.pg[0] - pa) < 1e-7
    assert abs(o.pg[1] - (pd - pa)) < 1e-7
    cost = 1e4 * (c2a * pa ** 2 + c2b * (pd - pa) ** 2)
    assert abs(o.cost - cost) < 1e-7 * cost


def test_lossless_dispatch_with_binding_pmax():
    net = _two_gen(0.02, 0.05, 1.4, pmax_a=0.6)
    o = opf.solve_opf(net, full_subsystem(net))
    assert o.status == opf.CONVERGED
    assert abs(o.pg[0] - 0.6) < 1e-7
    assert abs(o.pg[1] - 0.8) < 1e-7


def _ring(seed=0, rate=True):
    rng = np.random.default_rng(seed)
    n = 6
    br = [(k, (k + 1) % n, 0.01 + 0.02 * rng.random(), 0.05 + 0.1 * rng.random(),
           0.02 * rng.random()) for k in range(n)] + [(0, 3, 0.02, 0.1, 0.01)]
    gens = [dict(bus=0, pmax=3.0, c2=0.03), dict(bus=2, pmax=2.0, c2=0.06),
            dict(bus=4, pmax=2.0, c2=0.04)]
    loads = [(1, 0.9, 0.3), (3, 1.1, 0.4), (5, 0.7, 0.2)]
    net = make_net(n, br, gens, loads, rate=np.full(len(br), 1.0 if rate else 0.0))
    net["br_tap"][2] = 1.05           # exercise tap and phase shift
    net["br_shift"][2] = 0.03
    return net


def test_branch_admittance_matches_terminal_currents():
    """Y-bus from the pi model equals the currents computed terminal by
    terminal for an ideal transformer followed by the series impedance."""
    net = _ring()
    sub = full_subsystem(net)
    rng = np.random.default_rng(3)
    V = (1 + 0.05 * rng.standard_normal(6)) * np.exp(1j * 0.1 * rng.standard_normal(6))
    I = np.zeros(6, complex)
    for k in range(len(net["br_r"])):
        f, t = net["br_from"][k], net["br_to"][k]
        y = 1 / (net["br_r"][k] + 1j * net["br_x"][k])
        a = net["br_tap"][k] * np.exp(1j * net["br_shift"][k])
        vf_int = V[f] / a                     # ideal transformer secondary
        i_series = y * (vf_int - V[t])
        jb2 = 0.5j * net["br_b"][k]
        i_f_int = i_series + jb2 * vf_int
        I[f] += i_f_int / np.conj(a)          # power-conserving transformer
        I[t] += -i_series + jb2 * V[t]
    assert np.allclose(sub.Y @ V, I, rtol=0, atol=1e-12)


def test_jacobians_and_hessian_by_central_differences():
    net = _ring()
    sub = full_subsystem(net)
    P = opf.OPFProblem(net, sub)
    rng = np.random.default_rng(1)
    x = P.initial_point() + 0.05 * rng.standard_normal(P.nx)
    g, h, Jg, Jh, aux = P.evaluate(x)
    lam = rng.standard_normal(len(g))
    mu = rng.random(len(h))
    H = P.lagrangian_hessian(x, lam, mu, aux)
    eps = 1e-6
    for k in range(P.nx):
        e = np.zeros(P.nx)
        e[k] = eps
        gp, hp, Jgp, Jhp, _ = P.evaluate(x + e)
        gm, hm, Jgm, Jhm, _ = P.evaluate(x - e)
        assert np.allclose((gp - gm) / (2 * eps), Jg[:, k], atol=1e-6)
        assert np.allclose((hp - hm) / (2 * eps), Jh[:, k], atol=1e-6)
        Lp = P.cost_grad(x + e) + Jgp.T @ lam + Jhp.T @ mu
        Lm = P.cost_grad(x - e) + Jgm.T @ lam + Jhm.T @ mu
        assert np.allclose((Lp - Lm) / (2 * eps), H[:, k], atol=1e-5)
    assert np.allclose(H, H.T, atol=1e-10)


def test_kkt_certificate_at_optimum():
    net = _ring(rate=True)
    sub = full_subsystem(net)
    o = opf.solve_opf(net, sub)
    assert o.status == opf.CONVERGED
    P = opf.OPFProblem(net, sub)
    x = P.pack(o.va, o.vm, o.pg, o.qg)
    g, h, Jg, Jh, _ = P.evaluate(x)
    Lx = P.cost_grad(x) + Jg.T @ o.lam + Jh.T @ o.mu
    assert np.max(np.abs(g)) < 1e-8
    assert np.max(h) < 1e-8
    assert np.max(np.abs(Lx)) < 1e-8 * (1 + max(np.abs(o.lam).max(), o.mu.max()))
    assert np.all(o.mu >= 0) and np.all(o.z > 0)
    assert float(o.z @ o.mu) < 1e-7
    # ratings bind somewhere in this case, and the post-check agrees
    assert o.max_violation <= 1e-6


def test_rating_constraint_changes_dispatch():
    """Tight ratings must move the optimum (the flow block is active)."""
    a = _ring(rate=False)
    b = _ring(rate=False)
    b["br_rate"][:] = 0.53
    oa = opf.solve_opf(a, full_subsystem(a))
    ob = opf.solve_opf(b, full_subsystem(b))
    assert oa.status == ob.status == opf.CONVERGED
    assert ob.cost > oa.cost * (1 + 1e-6)
    sub = full_subsystem(b)
    V = ob.vm * np.exp(1j * ob.va)
    Sf = V[sub.f] * np.conj(sub.Yf @ V)
    St = V[sub.t] * np.conj(sub.Yt @ V)
    assert np.max(np.maximum(abs(Sf), abs(St))) <= 0.53 + 1e-7


def test_infeasible_load_is_not_converged():
    net = _two_bus(30.0, 5.0, 0.05, 0.3)
    o = opf.solve_opf(net, full_subsystem(net))
    assert o.status in (opf.MAXIT, opf.NUMERICAL)


@pytest.mark.parametrize("probe", [dict(kkt_solve="qr"), dict(row_scale_seed=1),
                                   dict(row_scale_seed=2)])
@pytest.mark.parametrize("rate", [True, False])
def test_rounding_probes_solve_the_same_steps(probe, rate):
    """The QR and row-scaled LU probes are exact reformulations of the Newton
    step: on a well-conditioned case they reach the same optimum in the same
    number of steps (only the last bits differ)."""
    net = _ring(rate=rate)
    sub = full_subsystem(net)
    ref = opf.solve_opf(net, sub)
    o = opf.solve_opf(net, sub, opf.OPFOptions(**probe))
    assert ref.status == o.status == opf.CONVERGED
    assert abs(o.iters - ref.iters) <= 1
    assert abs(o.cost - ref.cost) <= 1e-9 * abs(ref.cost)
    assert np.max(np.abs(o.vm - ref.vm)) < 1e-7
    assert np.max(np.abs(o.pg - ref.pg)) < 1e-7


def test_rounding_probe_changes_the_arithmetic():
    """The probes do change the rounding (else they would prove nothing)."""
    net = _ring(rate=True)
    sub = full_subsystem(net)
    ref = opf.solve_opf(net, sub)
    o = opf.solve_opf(net, sub, opf.OPFOptions(kkt_solve="qr"))
    assert not np.array_equal(o.vm, ref.vm) or not np.array_equal(o.pg, ref.pg)


def test_unknown_kkt_solve_rejected():
    net = _ring()
    with pytest.raises(ValueError):
        opf.solve_opf(net, full_subsystem(net), opf.OPFOptions(kkt_solve="cholesky"))
