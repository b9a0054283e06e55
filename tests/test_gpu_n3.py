"""N-3 screening with pruning on the device against the oracle
(tests/golden/c1_30_n3_oracle.npz: every triple of the 30-bus case's 41
branches, 10,660 rows, solved by the oracle, with its pruning flags and R_i).

* cs_screen_n3_device with the oracle's N-1/N-2 records as the screened
  list: the pruning flags equal the oracle's bit for bit, the solved rows'
  outcomes equal the oracle's to the bars of the other parity tests
  (helpers.outcome_mismatches), and R_i with pruned rows counted as severe
  within 1e-12 relative;
* cs_screen3_device on a mixed list (N-1 and N-2 rows padded with -1,
  triples): N-1/N-2 rows bit-identical to cs_screen_device of the same rows,
  triples equal to the oracle's records.
"""
import numpy as np
import pytest

from helpers import load_case, load_golden, outcome_mismatches

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_2512_08465_amd as cs
    ctx = cs.Context(0)
    case = load_case("c1_30")
    net = cs.Network(ctx, case)
    return cs, torch, ctx, case, net


def _records(cs, g):
    rec = np.zeros(len(g["severe"]), dtype=cs.RESULT_DTYPE)
    for k in ("severe", "cause", "opf_status", "near", "n_islands", "opf_iters", "n_states",
              "opf_cost", "max_real_eig", "min_damping", "max_violation"):
        rec[k] = g[k]
    return rec


def test_n3_with_pruning_matches_oracle(setup):
    cs, torch, ctx, case, net = setup
    g3 = load_golden("c1_30_n3")
    g2 = load_golden("c1_30")
    n3, n2 = len(g3["outages"]), len(g2["outages"])
    dev = torch.device("cuda:0")
    d_rows = torch.from_numpy(np.ascontiguousarray(g3["outages"], np.int32)).to(dev)
    d_sub = torch.from_numpy(np.ascontiguousarray(g2["outages"], np.int32)).to(dev)
    d_sub_rec = torch.from_numpy(_records(cs, g2).view(np.uint8).copy()).to(dev)
    d_lam = torch.from_numpy(case["lam"]).to(dev)
    d_out = torch.zeros(n3 * cs.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    d_R = torch.zeros(len(case["lam"]), dtype=torch.float64, device=dev)
    print(f"N-3: {n3} rows, {n2} screened sub-scenarios", flush=True)
    solved = net.screen_n3_device(d_rows.data_ptr(), n3, d_sub.data_ptr(), n2,
                                  d_sub_rec.data_ptr(), d_lam.data_ptr(), d_out.data_ptr(),
                                  d_R.data_ptr())
    res = d_out.cpu().numpy().view(cs.RESULT_DTYPE)
    R = d_R.cpu().numpy()
    keep = g3["keep"]
    pruned_dev = (res["cause"] & cs.CAUSE_PRUNED) > 0
    print(f"N-3: {int(keep.sum())} solved by the oracle's rule, {solved} on the device")
    assert solved == int(keep.sum())
    assert np.array_equal(pruned_dev, ~keep)
    assert np.all(res["severe"][~keep] == 1)
    bad, flips, kind = outcome_mismatches({k: g3[k][keep] for k in g3 if len(g3[k]) == n3},
                                          res[keep])
    print(f"N-3 solved rows: OPF converged on one side only {flips.tolist()}, both failed "
          f"with another kind {kind.tolist()}")
    assert len(bad) == 0, bad[:10]
    both = keep & (g3["opf_status"] == 0) & (res["opf_status"] == 0)
    rel = np.abs(res["opf_cost"][both] - g3["opf_cost"][both]) / np.abs(g3["opf_cost"][both])
    assert rel.max() < 1e-6
    # R_i: pruned rows count as severe
    touched = np.zeros(len(R), bool)
    sev_g = g3["severe"].astype(bool) | ~keep
    for i in np.flatnonzero(res["severe"].astype(bool) != sev_g):
        touched[[c for c in g3["outages"][i] if c >= 0]] = True
    ok = ~touched
    worst = np.max(np.abs(R[ok] - g3["risk_pruned"][ok]) / np.maximum(np.abs(g3["risk_pruned"][ok]),
                                                                        1e-300))
    print(f"N-3 R_i over {int(ok.sum())} components: worst relative {worst:.2e}")
    assert worst < 1e-12


def test_width3_rows_match_width2_and_oracle(setup):
    cs, torch, ctx, case, net = setup
    g3 = load_golden("c1_30_n3")
    g2 = load_golden("c1_30")
    rng = np.random.default_rng(3)
    i2 = np.sort(rng.choice(len(g2["outages"]), 120, replace=False))
    i3 = np.sort(rng.choice(len(g3["outages"]), 150, replace=False))
    rows2 = g2["outages"][i2]
    rows = np.concatenate([np.concatenate([rows2, np.full((len(rows2), 1), -1)], axis=1),
                           g3["outages"][i3], [[-1, -1, -1]]]).astype(np.int32)
    dev = torch.device("cuda:0")
    d_rows = torch.from_numpy(rows).to(dev)
    d_lam = torch.from_numpy(case["lam"]).to(dev)
    d_out = torch.zeros(len(rows) * cs.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    d_R = torch.zeros(len(case["lam"]), dtype=torch.float64, device=dev)
    net.screen3_device(d_rows.data_ptr(), len(rows), d_lam.data_ptr(), d_out.data_ptr(),
                       d_R.data_ptr())
    res = d_out.cpu().numpy().view(cs.RESULT_DTYPE)
    ref2, _ = net.screen(rows2, case["lam"])
    a = res[:len(rows2)]
    assert np.array_equal(a.view(np.uint8), ref2.view(np.uint8))
    sub = {k: g3[k][i3] for k in g3 if len(g3[k]) == len(g3["outages"])}
    bad, _, _ = outcome_mismatches(sub, res[len(rows2):-1])
    assert len(bad) == 0, bad[:10]
    # the base case row adds nothing; R_i is eq. (3) over the rows with the
    # N-3 frequency lambda_i lambda_j lambda_k
    from oracle import risk
    ref_R = risk.risk_index(rows, res["severe"], case["lam"], len(case["lam"]))
    assert np.allclose(d_R.cpu().numpy(), ref_R, rtol=1e-13, atol=0)


def test_width3_validation(setup):
    cs, torch, ctx, case, net = setup
    d_lam = torch.from_numpy(case["lam"]).cuda()
    d_out = torch.zeros(4 * cs.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    for bad in ([[1, 1, 2]], [[1, -1, 2]], [[1, 2, 200]], [[-1, 2, 3]], [[4, 5, 4]]):
        d = torch.tensor(bad, dtype=torch.int32, device="cuda")
        with pytest.raises(cs.CSError) as e:
            net.screen3_device(d.data_ptr(), 1, d_lam.data_ptr(), d_out.data_ptr(), None)
        assert e.value.code == cs.CS_EINVAL
