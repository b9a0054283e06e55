"""Serving (continuous batching) through the C-ABI: requests admitted into a
running server give, record for record, what cs_screen gives for the same
list alone, whether they run alone or overlap with other requests; the ring
refuses what does not fit (CS_EAGAIN) and a wait can time out."""
import threading

import numpy as np
import pytest

from helpers import load_case, load_golden

pytestmark = pytest.mark.gpu

FIELDS_EXACT = ("severe", "cause", "opf_status", "near", "n_islands", "opf_iters", "n_states")
FIELDS_FLOAT = ("opf_cost", "max_real_eig", "min_damping", "max_violation")


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_08465_amd as cs
    return cs.Context(0)


@pytest.fixture(scope="module")
def nets(ctx):
    import paper_2512_08465_amd as cs
    return {k: (cs.Network(ctx, load_case(k)), load_case(k)) for k in ("c1_30", "c2_118")}


def _same(a, b):
    for k in FIELDS_EXACT:
        assert np.array_equal(a[k], b[k]), k
    for k in FIELDS_FLOAT:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def _lists(name, sizes, seed):
    g = load_golden(name)["outages"]
    rng = np.random.default_rng(seed)
    return [g[np.sort(rng.choice(len(g), k, replace=False))] for k in sizes]


def test_requests_in_a_mix_equal_alone(nets):
    import paper_2512_08465_amd as cs
    net, case = nets["c1_30"]
    lists = _lists("c1_30", [120, 7, 300, 1, 55], seed=1)
    solo = [net.screen(l, case["lam"]) for l in lists]
    srv = cs.Server(net.ctx, net, cs.default_options(batch=64), queue_capacity=4096)
    reqs = [srv.submit(l, case["lam"]) for l in lists]
    for (res_s, risk_s), r in zip(solo, reqs):
        res, risk, lat = r.wait(timeout_s=100)
        _same(res, res_s)
        assert np.array_equal(risk, risk_s)
        assert lat > 0
    srv.close()


def test_arrivals_while_running_118(nets):
    """Requests submitted from another thread while earlier ones are on the
    device; the second network size runs in its own server at the same time."""
    import paper_2512_08465_amd as cs
    net, case = nets["c2_118"]
    net1, case1 = nets["c1_30"]
    lists = _lists("c2_118", [200, 40, 90], seed=2)
    lists1 = _lists("c1_30", [100, 100], seed=3)
    solo = [net.screen(l, case["lam"]) for l in lists]
    solo1 = [net1.screen(l, case1["lam"]) for l in lists1]
    srv = cs.Server(net.ctx, net, cs.default_options(batch=128), queue_capacity=1024)
    srv1 = cs.Server(net1.ctx, net1, cs.default_options(batch=32), queue_capacity=1024)
    reqs = [srv.submit(lists[0], case["lam"])]
    out = {}

    def later():
        out["r"] = [srv.submit(l, case["lam"]) for l in lists[1:]]
        out["r1"] = [srv1.submit(l, case1["lam"]) for l in lists1]

    t = threading.Thread(target=later)
    t.start()
    t.join()
    reqs += out["r"]
    for (res_s, risk_s), r in zip(solo, reqs):
        res, risk, _ = r.wait(timeout_s=100)
        _same(res, res_s)
        assert np.array_equal(risk, risk_s)
    for (res_s, risk_s), r in zip(solo1, out["r1"]):
        res, risk, _ = r.wait(timeout_s=100)
        _same(res, res_s)
        assert np.array_equal(risk, risk_s)
    srv.close()
    srv1.close()


def test_ring_full_and_timeout(nets):
    import paper_2512_08465_amd as cs
    net, case = nets["c2_118"]
    lists = _lists("c2_118", [60, 30], seed=4)
    srv = cs.Server(net.ctx, net, cs.default_options(batch=32), queue_capacity=80)
    r0 = srv.submit(lists[0], case["lam"])
    with pytest.raises(cs.CSError) as e:            # 60 + 30 > 80 positions
        srv.submit(lists[1], case["lam"])
    assert e.value.code == cs.CS_EAGAIN
    with pytest.raises(cs.CSError) as e:            # 60 scenarios of the 118-bus case
        r0.wait(timeout_s=0)
    assert e.value.code == cs.CS_ETIMEDOUT
    res0, _, _ = r0.wait(timeout_s=100)
    r1 = srv.submit(lists[1], case["lam"])          # room again
    res1, _, _ = r1.wait(timeout_s=100)
    _same(res0, net.screen(lists[0], case["lam"])[0])
    _same(res1, net.screen(lists[1], case["lam"])[0])
    with pytest.raises(cs.CSError) as e:
        srv.submit(np.array([[0, 0]]), case["lam"])
    assert e.value.code == cs.CS_EINVAL
    empty, risk, _ = srv.submit(np.zeros((0, 2), np.int32), case["lam"]).wait(timeout_s=1)
    assert len(empty) == 0 and np.all(risk == 0)
    srv.close()


def test_overlapped_streams_and_refill_equal(nets):
    """Two streams, and slots refilled many times over (batch much smaller
    than the list), give the same records as one stream with every scenario
    resident."""
    import paper_2512_08465_amd as cs
    net, case = nets["c2_118"]
    lst = _lists("c2_118", [300], seed=5)[0]
    a, Ra = net.screen(lst, case["lam"])
    b, Rb = net.screen(lst, case["lam"], cs.default_options(batch=48, overlap=1))
    c, Rc = net.screen(lst, case["lam"], cs.default_options(batch=100, overlap=0))
    # the second stream started only in the OPF tail, all slots resident and refilled
    d, Rd = net.screen(lst, case["lam"], cs.default_options(batch=300, overlap=2))
    f, Rf = net.screen(lst, case["lam"], cs.default_options(batch=64, overlap=2))
    _same(a, b)
    _same(a, c)
    _same(a, d)
    _same(a, f)
    assert np.array_equal(Ra, Rb) and np.array_equal(Ra, Rc)
    assert np.array_equal(Ra, Rd) and np.array_equal(Ra, Rf)


def _scaled_case(case, scale):
    c = dict(case)
    c["pd"] = case["pd"] * scale
    c["qd"] = case["qd"] * scale
    return c


def test_load_snapshots_equal_scaled_networks(nets):
    """Requests carrying their own load snapshot (every load times an N(1,
    0.05) factor), several in flight at once, give record for record what
    cs_screen gives on a network created with those loads; and the scaled
    network agrees with the oracle on the same snapshot."""
    import paper_2512_08465_amd as cs
    from inputs.rate_samples import load_scales
    from oracle import screen
    net, case = nets["c2_118"]
    nd = int(case["n_load"])
    scales = load_scales(nd, 3, seed=77)
    lists = _lists("c2_118", [40, 15, 60], seed=9)
    srv = cs.Server(net.ctx, net, cs.default_options(batch=48), queue_capacity=4096)
    reqs = [srv.submit(l, case["lam"], load_scale=s) for l, s in zip(lists, scales)]
    plain = srv.submit(lists[0], case["lam"])        # the network's own loads, in the mix
    got = []
    for l, s, r in zip(lists, scales, reqs):
        res, risk, _ = r.wait(timeout_s=300)
        got.append(res)
        snap = cs.Network(net.ctx, _scaled_case(case, s))
        ref, ref_risk = snap.screen(l, case["lam"])
        _same(res, ref)
        assert np.array_equal(risk, ref_risk)
        snap.close()
    res0, _, _ = plain.wait(timeout_s=300)
    ref0, _ = net.screen(lists[0], case["lam"])
    _same(res0, ref0)
    srv.close()
    # the snapshot itself against the oracle
    sc = _scaled_case(case, scales[0])
    for o, rec in zip(lists[0][:6], got[0][:6]):
        ref = screen.evaluate(sc, o)
        assert rec["n_islands"] == ref.n_islands
        if ref.opf_status == 0 and rec["opf_status"] == 0:
            assert abs(rec["opf_cost"] - ref.opf_cost) < 1e-6 * abs(ref.opf_cost)
            assert abs(rec["max_real_eig"] - ref.max_real_eig) < 1e-6 * max(1.0, abs(ref.max_real_eig))


def test_snapshot_factors_validated(nets):
    import paper_2512_08465_amd as cs
    net, case = nets["c1_30"]
    srv = cs.Server(net.ctx, net, cs.default_options(batch=16), queue_capacity=256)
    bad = np.ones(int(case["n_load"]))
    bad[2] = np.nan
    with pytest.raises(cs.CSError) as e:
        srv.submit(_lists("c1_30", [3], 1)[0], case["lam"], load_scale=bad)
    assert e.value.code == cs.CS_EINVAL
    srv.close()


def test_several_networks_one_budget(nets):
    """One server for the 30-, 118- and 300-bus networks under one HBM
    budget split by shares: requests for all three, interleaved and several
    in flight, give record for record what cs_screen gives for the same list
    on its network alone (a load snapshot included)."""
    import paper_2512_08465_amd as cs
    from inputs.rate_samples import load_scales
    net1, case1 = nets["c1_30"]
    net2, case2 = nets["c2_118"]
    case4 = load_case("c4_300")
    net4 = cs.Network(net2.ctx, case4)
    g4 = load_golden("c4_300")
    quick = np.flatnonzero(g4["opf_iters"] < 40)
    l4 = [g4["outages"][quick[:6]], g4["outages"][quick[6:16]]]
    l2 = _lists("c2_118", [70, 25], seed=21)
    l1 = _lists("c1_30", [90], seed=22)
    snap = load_scales(int(case2["n_load"]), 1, seed=23)[0]
    budget = 3 << 30
    srv = cs.Server(net2.ctx, [net1, net2, net4],
                    cs.default_options(batch=0, hbm_budget=budget), queue_capacity=2048,
                    shares=[1.0, 2.0, 4.0])
    s1, s2, s4 = srv.slots(0), srv.slots(1), srv.slots(2)
    print(f"slots under {budget >> 20} MiB split 1:2:4: 30-bus {s1}, 118-bus {s2}, 300-bus {s4}")
    assert 0 < s4 < s2
    reqs = [(4, l4[0], None, srv.submit(l4[0], case4["lam"], net=2)),
            (2, l2[0], None, srv.submit(l2[0], case2["lam"], net=1)),
            (1, l1[0], None, srv.submit(l1[0], case1["lam"], net=0)),
            (4, l4[1], None, srv.submit(l4[1], case4["lam"], net=2)),
            (2, l2[1], snap, srv.submit(l2[1], case2["lam"], load_scale=snap, net=1))]
    for kind, lst, sc, r in reqs:
        res, risk, lat = r.wait(timeout_s=600)
        if kind == 4:
            ref, ref_risk = net4.screen(lst, case4["lam"])
        elif kind == 1:
            ref, ref_risk = net1.screen(lst, case1["lam"])
        elif sc is None:
            ref, ref_risk = net2.screen(lst, case2["lam"])
        else:
            snap_net = cs.Network(net2.ctx, _scaled_case(case2, sc))
            ref, ref_risk = snap_net.screen(lst, case2["lam"])
            snap_net.close()
        print(f"{kind}: {len(lst)} scenarios, latency {lat:.2f} s")
        _same(res, ref)
        assert np.array_equal(risk, ref_risk)
    with pytest.raises(cs.CSError) as e:
        srv.submit(l1[0], case1["lam"], net=3)
    assert e.value.code == cs.CS_EINVAL
    srv.close()
    with pytest.raises(cs.CSError) as e:
        cs.Server(net2.ctx, [net1, net2], shares=[1.0, 0.0])
    assert e.value.code == cs.CS_EINVAL
    net4.close()


def test_overlap_with_islanding_only_lists(nets):
    """Two streams with a batch of at most 1,024 slots claim every slot for
    the dynamic stage at once; when the claimed scenarios need little
    dynamic work (islanded, most with a failed OPF) the stage can finish
    between the engine's query and its stage counts.  The engine asks first,
    so the call finishes; records equal the one-stream run's, in a batch call
    and in a server."""
    import paper_2512_08465_amd as cs
    net, case = nets["c1_30"]
    g = load_golden("c1_30")
    isl = g["outages"][g["n_islands"] > 1]
    assert len(isl) >= 20
    lst = np.concatenate([isl] * 4)
    print(f"{len(lst)} islanding scenarios, batch 16, two streams", flush=True)
    ref, ref_r = net.screen(lst, case["lam"], cs.default_options(batch=16))
    got, got_r = net.screen(lst, case["lam"], cs.default_options(batch=16, overlap=1))
    _same(got, ref)
    assert np.array_equal(got_r, ref_r)
    got, got_r = net.screen(lst, case["lam"], cs.default_options(batch=16, overlap=2))
    _same(got, ref)
    assert np.array_equal(got_r, ref_r)
    srv = cs.Server(net.ctx, net, cs.default_options(batch=16, overlap=1), queue_capacity=1024)
    reqs = [srv.submit(lst[i::3], case["lam"]) for i in range(3)]
    for i, r in enumerate(reqs):
        res, risk, _ = r.wait(timeout_s=300)
        _same(res, ref[i::3])
    srv.close()
