"""Mixed precision (FP32 KKT factorisation on the matrix cores + FP64
refinement, FP64 fallback) against the oracle's stored records, to the same
bars as the FP64 path, and against the FP64 GPU path.  The largest deviations
from the oracle are printed (pytest -s) for the record."""
import numpy as np
import pytest

from helpers import load_case, load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_08465_amd as cs
    return cs.Context(0)


@pytest.fixture(scope="module")
def runs(ctx):
    import paper_2512_08465_amd as cs
    out = {}
    for name in ("c1_30", "c2_118", "c3_118", "c4_300"):
        case = load_case(name)
        g = load_golden(name)
        net = cs.Network(ctx, case)
        ctx.reset_stats()
        mixed = net.screen(g["outages"], case["lam"],
                           cs.default_options(prec=cs.PREC_MIXED, timing=1))
        st = ctx.stats()
        plain = net.screen(g["outages"], case["lam"])
        out[name] = (g, mixed, plain, st)
    return out


@pytest.mark.parametrize("name", ["c1_30", "c2_118", "c3_118", "c4_300"])
def test_mixed_matches_oracle(runs, name):
    from helpers import outcome_mismatches, rounding_listed
    g, (res, R), _, st = runs[name]
    flip_ok = rounding_listed(g["outages"]) if name in ("c2_118", "c3_118") else []
    bad, flips, kind = outcome_mismatches(g, res, flip_ok)
    print(f"\n{name} mixed: OPF converged on one side only {flips.tolist()}, both failed "
          f"with another kind {kind.tolist()}")
    assert len(bad) == 0, bad[:10]
    both = (g["opf_status"] == 0) & (res["opf_status"] == 0)
    rel_cost = np.abs(res["opf_cost"][both] - g["opf_cost"][both]) / np.abs(g["opf_cost"][both])
    d_alpha = np.abs(res["max_real_eig"][both] - g["max_real_eig"][both]) / \
        np.maximum(np.abs(g["max_real_eig"][both]), 1.0)
    d_zeta = np.abs(res["min_damping"][both] - g["min_damping"][both])
    print(f"\n{name} mixed vs oracle: cost rel {rel_cost.max():.2e}, max Re rel "
          f"{d_alpha.max():.2e}, damping {d_zeta.max():.2e}; FP64 fallbacks "
          f"{st['kkt_lu64']['units']} of {st['kkt_lu']['units']} KKT solves")
    assert rel_cost.max() < 1e-6
    assert d_alpha.max() < 1e-6
    assert d_zeta.max() < 1e-6
    assert np.array_equal(res["n_states"][both], g["n_states"][both])
    listed = np.zeros(len(res), bool)
    if name in ("c2_118", "c3_118"):
        listed[rounding_listed(g["outages"], ("outcome", "path"))] = True
    dit = np.abs(res["opf_iters"].astype(int) - g["opf_iters"])
    assert np.all(dit[both & ~listed] <= 2), np.flatnonzero(both & ~listed & (dit > 2))
    assert st["kkt_lu"]["units"] > 0


@pytest.mark.parametrize("name", ["c1_30", "c2_118", "c3_118", "c4_300"])
def test_mixed_matches_fp64_path(runs, name):
    _, (res, R), (ref, Rref), _ = runs[name]
    conv = ref["opf_status"] == 0
    same = conv & (res["opf_status"] == 0)
    assert same.sum() >= 0.98 * conv.sum()
    rel = np.abs(res["opf_cost"][same] - ref["opf_cost"][same]) / np.abs(ref["opf_cost"][same])
    print(f"\n{name} mixed vs FP64 GPU: cost rel {rel.max():.2e}")
    assert rel.max() < 1e-7
    from helpers import outcome_mismatches, rounding_listed
    flip_ok = rounding_listed(load_golden(name)["outages"]) if name in ("c2_118", "c3_118") \
        else []
    bad, _, _ = outcome_mismatches(ref, res, flip_ok)
    assert len(bad) == 0, bad[:10]
