"""Risk Index extensions on the device against the oracle (oracle/risk.py),
from the same records (the oracle's stored records of the whole 118-bus-shaped
list and of the 30-bus list), so that only the risk arithmetic is compared:

* non-binary (damping-based) severity and common-cause pairs (cs_risk):
  R_i within 1e-12 relative, bit-identical run to run, and the binary,
  independent case equal to eq. (3);
* Monte-Carlo over seeded log-normal failure-rate samples (cs_risk_mc): every
  sample's R_i within 1e-12 relative (largest entry of the sample), mean and
  standard deviation within 1e-12, rank histograms and rank quantiles exact
  except where two components' R lie within 1e-12 of each other in a sample
  (ranks decided by rounding; then the device's ranks are checked to be a
  valid ordering of the oracle's values).
"""
import numpy as np
import pytest

from helpers import load_case, load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_08465_amd as cs
    return cs.Context(0)


def _records(cs, g):
    rec = np.zeros(len(g["severe"]), dtype=cs.RESULT_DTYPE)
    for k in ("severe", "cause", "opf_status", "near", "n_islands", "opf_iters", "n_states",
              "opf_cost", "max_real_eig", "min_damping", "max_violation"):
        rec[k] = g[k]
    return rec


@pytest.fixture(scope="module", params=["c1_30", "c2_118_full"])
def setup(request, ctx):
    import torch
    import paper_2512_08465_amd as cs
    name = request.param
    case = load_case("c2_118" if name == "c2_118_full" else name)
    g = load_golden(name)
    net = cs.Network(ctx, case)
    rec = _records(cs, g)
    dev = torch.device("cuda:0")
    d = dict(out=torch.from_numpy(np.ascontiguousarray(g["outages"], np.int32)).to(dev),
             rec=torch.from_numpy(rec.view(np.uint8).copy()).to(dev),
             lam=torch.from_numpy(case["lam"]).to(dev))
    return name, case, g, net, d


CC = [[0, 5], [3, 17], [0, 5], [12, 40]]
CC_RATE = [0.02, 0.005, 0.01, 0.0]


@pytest.mark.parametrize("mode,cc", [(0, False), (1, False), (0, True), (1, True)])
def test_risk_variants_match_oracle(setup, mode, cc):
    import torch
    from oracle import risk
    name, case, g, net, d = setup
    n_comp = len(case["lam"])
    n = len(g["severe"])
    w = risk.severity_weights(g["severe"], g["min_damping"], mode, 0.05)
    table = risk.common_cause_table(CC, CC_RATE, n_comp) if cc else None
    ref = risk.risk_index_weighted(g["outages"], w, case["lam"], n_comp, table)
    out = []
    for _ in range(2):
        d_r = torch.full((n_comp,), -1.0, dtype=torch.float64, device="cuda")
        net.risk(d["out"].data_ptr(), n, d["rec"].data_ptr(), d["lam"].data_ptr(),
                 d_r.data_ptr(), severity=mode, zeta_ref=0.05,
                 cc_pairs=CC if cc else None, cc_rate=CC_RATE if cc else None)
        out.append(d_r.cpu().numpy())
    assert np.array_equal(out[0].view(np.uint64), out[1].view(np.uint64))
    scale = np.maximum(np.abs(ref), 1e-300)
    worst = float(np.max(np.abs(out[0] - ref) / scale))
    print(f"{name} severity mode {mode} cc {cc}: worst relative {worst:.2e}")
    assert worst < 1e-12
    if mode == 0 and not cc:
        # the binary, independent case is eq. (3) over the records
        assert np.allclose(out[0], g["risk"], rtol=1e-12, atol=0)
    if mode == 1:
        assert np.all(out[0] >= risk.risk_index_weighted(
            g["outages"], np.asarray(g["severe"], float), case["lam"], n_comp, table) - 1e-15)


@pytest.mark.parametrize("mode,cc", [(0, False), (1, True)])
def test_monte_carlo_matches_oracle(setup, mode, cc):
    import torch
    from oracle import risk
    from inputs.rate_samples import lognormal_rates
    name, case, g, net, d = setup
    n_comp = len(case["lam"])
    n = len(g["severe"])
    M = 48 if name == "c2_118_full" else 300
    S = lognormal_rates(case["lam"], M, sigma=0.5, seed=77)
    w = risk.severity_weights(g["severe"], g["min_damping"], mode, 0.05)
    table = risk.common_cause_table(CC, CC_RATE, n_comp) if cc else None
    R, mean, std, hist, quant = risk.risk_monte_carlo(g["outages"], w, S, n_comp, table)
    d_S = torch.from_numpy(S).cuda()
    d_R = torch.zeros((M, n_comp), dtype=torch.float64, device="cuda")
    d_mom = torch.zeros((n_comp, 2), dtype=torch.float64, device="cuda")
    d_q = torch.zeros((n_comp, 3), dtype=torch.int32, device="cuda")
    print(f"{name}: Monte-Carlo with {M} samples", flush=True)
    net.risk_mc(d["out"].data_ptr(), n, d["rec"].data_ptr(), d_S.data_ptr(), M,
                d_R.data_ptr(), d_mom.data_ptr(), d_q.data_ptr(), severity=mode, zeta_ref=0.05,
                cc_pairs=CC if cc else None, cc_rate=CC_RATE if cc else None)
    Rd, mom, q = d_R.cpu().numpy(), d_mom.cpu().numpy(), d_q.cpu().numpy()
    scale = np.max(np.abs(R), axis=1, keepdims=True)
    dev_R = float(np.max(np.abs(Rd - R) / scale))
    dev_m = float(np.max(np.abs(mom[:, 0] - mean) / np.max(np.abs(mean))))
    dev_s = float(np.max(np.abs(mom[:, 1] - std) / np.max(np.abs(std))))
    print(f"{name}: R {dev_R:.2e}, mean {dev_m:.2e}, std {dev_s:.2e}")
    assert dev_R < 1e-12 and dev_m < 1e-12 and dev_s < 1e-12
    # components whose rank rounding may decide: a near tie in some sample
    tie = np.zeros(n_comp, bool)
    for m in range(M):
        o = np.argsort(-R[m], kind="stable")
        gap = np.abs(np.diff(R[m][o])) <= 1e-12 * scale[m, 0]
        gap &= ~((R[m][o][:-1] == R[m][o][1:]))       # exact ties: id order on both sides
        tie[o[:-1][gap]] = True
        tie[o[1:][gap]] = True
    bad = np.flatnonzero(~tie & np.any(q != quant, axis=1))
    print(f"{name}: {int(tie.sum())} components with a near tie; quantile mismatches {bad.tolist()}")
    assert len(bad) == 0
    # the device's ranks, recomputed from its own R, are a valid ordering
    for m in range(0, M, max(1, M // 8)):
        o = np.lexsort((np.arange(n_comp), -Rd[m]))
        assert np.all(np.diff(R[m][o]) <= 1e-12 * scale[m, 0])


def test_risk_options_rejected(setup):
    import torch
    import paper_2512_08465_amd as cs
    name, case, g, net, d = setup
    n_comp = len(case["lam"])
    d_r = torch.zeros(n_comp, dtype=torch.float64, device="cuda")
    args = (d["out"].data_ptr(), 10, d["rec"].data_ptr(), d["lam"].data_ptr(), d_r.data_ptr())
    for kw in (dict(severity=3), dict(severity=1, zeta_ref=0.0),
               dict(cc_pairs=[[1, 1]], cc_rate=[0.1]), dict(cc_pairs=[[1, n_comp]], cc_rate=[0.1]),
               dict(cc_pairs=[[1, 2]], cc_rate=[-0.1])):
        with pytest.raises(cs.CSError) as e:
            net.risk(*args, **kw)
        assert e.value.code == cs.CS_EINVAL, kw
    bad = torch.from_numpy(case["lam"]).cuda().reshape(1, -1).clone()
    bad[0, 3] = float("nan")
    with pytest.raises(cs.CSError) as e:
        net.risk_mc(d["out"].data_ptr(), 10, d["rec"].data_ptr(), bad.data_ptr(), 1,
                    d_r.data_ptr())
    assert e.value.code == cs.CS_EINVAL
