"""Error paths and forced conditions of the screening call, each forced from
the host so that every kernel still runs to its normal end.

* a workspace budget below one scenario's need is rejected (CS_EHBM);
* an iteration cap of one step leaves every OPF unconverged: each scenario
  is severe for OPF non-convergence (Section II.B.1), none is linearised;
* a non-finite value in the network is rejected at creation (CS_EINVAL);
* the mixed-precision solve with no refinement step allowed sends every
  Newton system to the FP64 factorisation, and the records equal the FP64
  path's (the fallback is the FP64 solve itself);
* bad options are rejected before any device work.
"""
import numpy as np
import pytest

from helpers import load_case, load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_08465_amd as cs
    return cs.Context(0)


@pytest.fixture(scope="module")
def c1(ctx):
    import paper_2512_08465_amd as cs
    return cs.Network(ctx, load_case("c1_30"))


def test_budget_below_one_scenario_is_rejected(ctx, c1):
    import paper_2512_08465_amd as cs
    g = load_golden("c1_30")
    with pytest.raises(cs.CSError) as e:
        c1.screen(g["outages"][:4], None, cs.default_options(hbm_budget=4096))
    assert e.value.code == cs.CS_EHBM
    small = cs.Context(0, hbm_budget=4096)
    net = cs.Network(small, load_case("c1_30"))
    with pytest.raises(cs.CSError) as e:
        net.screen(g["outages"][:4])
    assert e.value.code == cs.CS_EHBM
    with pytest.raises(cs.CSError) as e:
        cs.Server(small, net, cs.default_options(), queue_capacity=64)
    assert e.value.code == cs.CS_EHBM
    # the budget of exactly one slot still screens (one slot, refilled)
    res, _ = c1.screen(g["outages"][:3], None, cs.default_options(batch=1))
    assert np.array_equal(res["n_islands"], g["n_islands"][:3])


def test_iteration_cap_of_one_step(c1):
    import paper_2512_08465_amd as cs
    g = load_golden("c1_30")
    lst = g["outages"][:60]
    res, R = c1.screen(lst, load_case("c1_30")["lam"], cs.default_options(max_it=1))
    ran = res["opf_status"] != cs.OPF_NOT_RUN
    assert ran.sum() > 0
    assert np.all(res["opf_status"][ran] != cs.OPF_CONVERGED)
    assert np.all(res["opf_iters"][ran] <= 1)
    assert np.all(res["severe"] == 1)
    assert np.all(res["cause"] & cs.CAUSE_OPF)
    assert np.all(res["n_states"] == 0)
    assert np.all(np.isnan(res["max_real_eig"]))
    assert np.array_equal(res["n_islands"], g["n_islands"][:60])
    # every scenario severe: R_i is the whole of eq. (3) over the list
    lam = load_case("c1_30")["lam"]
    ref = np.zeros_like(lam)
    for a, b in lst:
        f = lam[a] if b < 0 else lam[a] * lam[b]
        ref[a] += f
        if b >= 0:
            ref[b] += f
    assert np.allclose(R, ref, rtol=1e-13, atol=0)


def test_non_finite_network_is_rejected(ctx):
    import paper_2512_08465_amd as cs
    for key, idx in (("br_x", 3), ("pd", 0), ("dyn", (2, 5)), ("vmax", 7)):
        case = load_case("c1_30")
        case[key] = case[key].copy()
        case[key][idx] = np.nan
        with pytest.raises(cs.CSError) as e:
            cs.Network(ctx, case)
        assert e.value.code == cs.CS_EINVAL, key
    case = load_case("c1_30")
    case["br_r"] = case["br_r"].copy()
    case["br_r"][1] = np.inf
    with pytest.raises(cs.CSError) as e:
        cs.Network(ctx, case)
    assert e.value.code == cs.CS_EINVAL


def test_mixed_without_refinement_falls_back_to_fp64(ctx, c1):
    import paper_2512_08465_amd as cs
    g = load_golden("c1_30")
    lst = g["outages"][:120]
    ctx.reset_stats()
    mixed, _ = c1.screen(lst, None, cs.default_options(prec=cs.PREC_MIXED, refine_steps=0,
                                                       timing=1))
    st = ctx.stats()
    n_ran = int((mixed["opf_iters"] > 0).sum())
    assert n_ran > 0
    # every scenario's first FP32 solve fails its backward-error test; the
    # scenario then stays on FP64 factorisations for the rest of its OPF
    assert 0 < st["kkt_lu"]["units"] <= n_ran
    assert st["kkt_lu64"]["units"] >= int(mixed["opf_iters"].sum()) - n_ran
    plain, _ = c1.screen(lst, None)
    for k in ("severe", "cause", "opf_status", "opf_iters", "n_islands", "n_states"):
        assert np.array_equal(mixed[k], plain[k]), k
    for k in ("opf_cost", "max_real_eig", "min_damping"):
        assert np.array_equal(mixed[k], plain[k], equal_nan=True), k
    # with refinement allowed, solves stay in FP32 for several steps
    ctx.reset_stats()
    c1.screen(lst, None, cs.default_options(prec=cs.PREC_MIXED, timing=1))
    st = ctx.stats()
    assert st["kkt_lu"]["units"] > 2 * n_ran


@pytest.mark.parametrize("field,value", [("prec", 7), ("max_it", 0), ("tol", 0.0),
                                         ("refine_steps", -1), ("refine_steps", 101),
                                         ("graph", -1), ("graph", 65), ("autotune", 2),
                                         ("overlap", -1), ("overlap", 3)])
def test_bad_options_rejected(c1, field, value):
    import paper_2512_08465_amd as cs
    with pytest.raises(cs.CSError) as e:
        c1.screen(np.array([[0, -1]]), None, cs.default_options(**{field: value}))
    assert e.value.code == cs.CS_EINVAL


def test_context_destroyed_before_its_network(c1):
    """Destroying a context before its network (the C order, or a garbage
    collector finalising both) leaves no error behind for later calls."""
    import gc
    import paper_2512_08465_amd as cs
    case = load_case("c1_30")
    ctx2 = cs.Context(0)
    net2 = cs.Network(ctx2, case)
    ctx2.close()                        # closes net2 first
    assert not net2._h
    ctx3 = cs.Context(0)
    net3 = cs.Network(ctx3, case)
    cs.library().cs_ctx_destroy(ctx3._h)  # the C order: context first
    ctx3._h = type(ctx3._h)()
    net3.close()
    del net2, net3, ctx2, ctx3
    gc.collect()
    g = load_golden("c1_30")
    res, _ = c1.screen(g["outages"][:5])
    assert np.array_equal(res["n_islands"], g["n_islands"][:5])
