"""Pins for the oracle's per-scenario severity rules (Section II.B).

Each criterion of Section II.B is exercised on a hand-built network whose
outcome is known without the oracle: a radial branch taken out leaves an
island (II.B.3); a load beyond every generator's capacity has no feasible OPF
(II.B.1); with every generator out there is nothing to solve (II.B.3, main
island without generation); a machine with negative damping has a growing
electromechanical mode (II.B.2).  The decision rules themselves are checked
at their exact thresholds: Re(lambda) >= 0 is inclusive, the limit test is a
strict excess over 1e-6 p.u., and each near-threshold flag sits on its band.
"""
import math

import numpy as np
import pytest

from oracle import screen, opf
from nets import make_net, base_dyn_row

CONV, MAXIT, NUMERICAL, NOT_RUN = opf.CONVERGED, opf.MAXIT, opf.NUMERICAL, opf.NOT_RUN
up = lambda v: math.nextafter(v, math.inf)      # noqa: E731
down = lambda v: math.nextafter(v, -math.inf)   # noqa: E731


def _meshed_with_radial_bus():
    """Buses 0-2 in a triangle, bus 3 hangs off bus 2 (branch 3 is a bridge).
    Generators at buses 0 and 1, loads at buses 2 and 3."""
    br = [(0, 1, 0.01, 0.08, 0.02), (1, 2, 0.01, 0.1, 0.02), (0, 2, 0.02, 0.12, 0.01),
          (2, 3, 0.01, 0.06, 0.01)]
    gens = [dict(bus=0, pmax=2.0, c2=0.02), dict(bus=1, pmax=1.5, c2=0.04)]
    loads = [(2, 0.8, 0.2), (3, 0.4, 0.1)]
    return make_net(4, br, gens, loads, vmin=0.9, vmax=1.1)


def test_radial_branch_outage_islands():
    net = _meshed_with_radial_bus()
    r = screen.evaluate(net, np.array([3, -1]))
    assert r.n_islands == 2
    assert r.cause & screen.CAUSE_ISLAND
    assert r.severe == 1
    # the island with the generation is still solved
    assert r.opf_status == CONV
    # a branch of the triangle is not a bridge: no island, a secure scenario
    r = screen.evaluate(net, np.array([0, -1]))
    assert r.n_islands == 1 and r.cause == 0 and r.severe == 0


def test_load_beyond_capacity_fails_the_opf():
    """Two buses, one generator of 0.5 p.u. feeding a 1.0 p.u. load: no
    feasible dispatch exists, so the OPF cannot converge."""
    net = make_net(2, [(0, 1, 0.01, 0.1, 0.0)], [dict(bus=0, pmax=0.5, c2=0.05)],
                   [(1, 1.0, 0.2)])
    r = screen.evaluate(net, np.array([-1, -1]), screen.ScreenOptions(max_it=60))
    assert r.opf_status in (MAXIT, NUMERICAL)
    assert r.cause & screen.CAUSE_OPF
    assert bool(r.cause & screen.CAUSE_NUMERICAL) == (r.opf_status == NUMERICAL)
    assert r.severe == 1
    assert r.n_states == 0 and math.isnan(r.max_real_eig)


def test_every_generator_out_is_not_run():
    net = _meshed_with_radial_bus()
    nl = int(net["n_branch"])
    r = screen.evaluate(net, np.array([nl, nl + 1]))
    assert r.opf_status == NOT_RUN
    assert r.n_islands == 1
    assert r.cause == screen.CAUSE_OPF
    assert r.severe == 1
    assert r.opf_iters == 0 and math.isnan(r.opf_cost)
    # one generator left: solved
    r = screen.evaluate(net, np.array([nl, -1]))
    assert r.opf_status == CONV


def _pair(D1):
    row0 = base_dyn_row(D=2.0)
    row1 = base_dyn_row(D=D1)
    gens = [dict(bus=0, pmax=2.0, c2=0.02, dyn=row0), dict(bus=1, pmax=2.0, c2=0.03, dyn=row1)]
    return make_net(3, [(0, 1, 0.01, 0.1, 0.01), (1, 2, 0.01, 0.1, 0.01), (0, 2, 0.02, 0.15, 0.0)],
                    gens, [(2, 1.2, 0.3)])


def test_negative_damping_is_small_signal_unstable():
    """A machine whose damping torque opposes its speed deviation
    (D well below zero) has an electromechanical mode with positive real part."""
    stable = screen.evaluate(_pair(2.0), np.array([-1, -1]))
    assert stable.opf_status == CONV
    assert stable.max_real_eig < 0 and not stable.cause & screen.CAUSE_SSS
    r = screen.evaluate(_pair(-60.0), np.array([-1, -1]))
    assert r.opf_status == CONV
    assert r.max_real_eig > 0
    assert r.cause == screen.CAUSE_SSS and r.severe == 1


@pytest.mark.parametrize("alpha,severe", [(0.0, True), (-0.0, True), (5e-324, True),
                                          (-5e-324, False), (-1.0, False), (3.0, True)])
def test_real_part_test_is_inclusive(alpha, severe):
    c = screen.classify(1, CONV, -1.0, alpha)
    assert bool(c & screen.CAUSE_SSS) == severe
    assert c in (0, screen.CAUSE_SSS)


@pytest.mark.parametrize("viol,severe", [(1e-6, False), (up(1e-6), True), (-0.2, False),
                                         (0.0, False), (0.3, True)])
def test_limit_test_is_a_strict_excess(viol, severe):
    c = screen.classify(1, CONV, viol, -1.0)
    assert bool(c & screen.CAUSE_LIMIT) == severe
    assert c in (0, screen.CAUSE_LIMIT)


def test_cause_bits_by_outcome():
    nan = float("nan")
    assert screen.classify(2, CONV, -1.0, -1.0) == screen.CAUSE_ISLAND
    assert screen.classify(1, MAXIT, nan, nan) == screen.CAUSE_OPF
    assert screen.classify(1, NUMERICAL, nan, nan) == screen.CAUSE_OPF | screen.CAUSE_NUMERICAL
    assert screen.classify(3, NOT_RUN, nan, nan) == screen.CAUSE_OPF | screen.CAUSE_ISLAND
    # a non-finite state matrix is a numerical failure, not an SSS verdict
    assert screen.classify(1, CONV, -1.0, nan, state_finite=False) == screen.CAUSE_NUMERICAL
    # every criterion at once
    assert screen.classify(2, CONV, 1.0, 0.5) == (screen.CAUSE_ISLAND | screen.CAUSE_LIMIT
                                                   | screen.CAUSE_SSS)


def test_near_flags_on_their_bands():
    o = screen.ScreenOptions()          # max_it 150, near_eps 1e-6
    nf = screen.near_flags
    # OPF: converged within two steps of the cap
    assert nf(CONV, 148, -1.0, -1.0, o) == screen.NEAR_OPF
    assert nf(CONV, 150, -1.0, -1.0, o) == screen.NEAR_OPF
    assert nf(CONV, 147, -1.0, -1.0, o) == 0
    # a run that hit the cap is not itself near (both sides reaching the cap agree)
    assert nf(MAXIT, 150, float("nan"), float("nan"), o) == 0
    assert nf(NUMERICAL, 149, float("nan"), float("nan"), o) == 0
    # limit: a decade either side of 1e-6 p.u.
    for v, flag in [(1e-7, 0), (up(1e-7), screen.NEAR_LIMIT), (1e-6, screen.NEAR_LIMIT),
                    (1e-5, screen.NEAR_LIMIT), (up(1e-5), 0), (0.3, 0), (-1e-3, 0)]:
        assert nf(CONV, 20, v, -1.0, o) == flag, v
    # SSS: |max Re| within near_eps of zero
    for a, flag in [(1e-6, screen.NEAR_SSS), (-1e-6, screen.NEAR_SSS), (0.0, screen.NEAR_SSS),
                    (up(1e-6), 0), (down(-1e-6), 0)]:
        assert nf(CONV, 20, -1.0, a, o) == flag, a
    # near_eps is an option
    assert nf(CONV, 20, -1.0, -1e-4, screen.ScreenOptions(near_eps=1e-3)) == screen.NEAR_SSS
    # iteration cap is an option
    assert nf(CONV, 18, -1.0, -1.0, screen.ScreenOptions(max_it=20)) == screen.NEAR_OPF


def test_evaluate_applies_the_rules():
    """The record's bits are the rules applied to the record's own values."""
    for net, out in [(_meshed_with_radial_bus(), [3, -1]), (_pair(-60.0), [-1, -1]),
                     (_pair(2.0), [-1, -1]), (_meshed_with_radial_bus(), [4, 5])]:
        r = screen.evaluate(net, np.array(out))
        assert r.cause == screen.classify(r.n_islands, r.opf_status, r.max_violation,
                                          r.max_real_eig)
        assert r.near == screen.near_flags(r.opf_status, r.opf_iters, r.max_violation,
                                           r.max_real_eig)
        assert r.severe == int(r.cause != 0)
