"""The allocation-free screening entry point (cs_screen_device_noalloc)
against the ordinary device entry point (cs_screen_device): the same records
and Risk Index, bit for bit (a scenario's arithmetic does not depend on the
slot it runs in), on two calls in a row, the second with a shorter list, and
on two network sizes.  Timing, which allocates, is refused."""
import numpy as np
import pytest

from helpers import load_case, load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_08465_amd as cs
    return cs.Context(0)


def _both(cs, torch, net, lam, lst):
    dev = torch.device("cuda:0")
    n = len(lst)
    rec = cs.RESULT_DTYPE.itemsize
    d_list = torch.from_numpy(np.ascontiguousarray(lst, dtype=np.int32)).to(dev)
    d_lam = torch.from_numpy(lam).to(dev)
    out = []
    for noalloc in (False, True):
        d_res = torch.full((max(n, 1) * rec,), 0xAB, dtype=torch.uint8, device=dev)
        d_risk = torch.full((len(lam),), -1.0, dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        torch.cuda.synchronize()
        f = net.screen_device_noalloc if noalloc else net.screen_device
        print(f"{'noalloc' if noalloc else 'device'}: {n} scenarios", flush=True)
        f(d_list.data_ptr(), n, d_lam.data_ptr(), d_res.data_ptr(), d_risk.data_ptr(),
          stream=stream)
        torch.cuda.synchronize()
        out.append((d_res.cpu().numpy()[:n * rec].view(cs.RESULT_DTYPE), d_risk.cpu().numpy()))
    return out


@pytest.mark.parametrize("name,first,second", [("c2_118", 260, 90), ("c1_30", 861, 200)])
def test_noalloc_matches_device_entry_point(ctx, name, first, second):
    import torch
    import paper_2512_08465_amd as cs
    case = load_case(name)
    g = load_golden(name)
    net = cs.Network(ctx, case)
    rng = np.random.default_rng(11)
    lst1 = g["outages"][rng.permutation(len(g["outages"]))[:first]]
    lst2 = g["outages"][rng.permutation(len(g["outages"]))[:second]]
    for lst in (lst1, lst2):
        (ra, Ra), (rb, Rb) = _both(cs, torch, net, case["lam"], lst)
        assert np.array_equal(ra.view(np.uint8), rb.view(np.uint8))
        assert np.array_equal(Ra.view(np.uint64), Rb.view(np.uint64))
        assert np.array_equal(ra["n_islands"], g["n_islands"][
            [int(np.flatnonzero((g["outages"] == o).all(1))[0]) for o in lst]])


def test_noalloc_refuses_timing_and_bad_rows(ctx):
    import torch
    import paper_2512_08465_amd as cs
    case = load_case("c1_30")
    net = cs.Network(ctx, case)
    dev = torch.device("cuda:0")
    d_lam = torch.from_numpy(case["lam"]).to(dev)
    d_res = torch.zeros(4 * cs.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    d_risk = torch.zeros(len(case["lam"]), dtype=torch.float64, device=dev)
    good = torch.tensor([[0, -1], [1, 2]], dtype=torch.int32, device=dev)
    with pytest.raises(cs.CSError) as e:
        net.screen_device_noalloc(good.data_ptr(), 2, d_lam.data_ptr(), d_res.data_ptr(),
                                  d_risk.data_ptr(), cs.default_options(timing=1))
    assert e.value.code == cs.CS_EINVAL
    bad = torch.tensor([[0, -1], [3, 3]], dtype=torch.int32, device=dev)
    with pytest.raises(cs.CSError) as e:
        net.screen_device_noalloc(bad.data_ptr(), 2, d_lam.data_ptr(), d_res.data_ptr(),
                                  d_risk.data_ptr())
    assert e.value.code == cs.CS_EINVAL
    neg = d_lam.clone()
    neg[5] = -0.5
    with pytest.raises(cs.CSError) as e:
        net.screen_device_noalloc(good.data_ptr(), 2, neg.data_ptr(), d_res.data_ptr(),
                                  d_risk.data_ptr())
    assert e.value.code == cs.CS_EINVAL
    # an empty list: R_i = 0
    net.screen_device_noalloc(good.data_ptr(), 0, d_lam.data_ptr(), d_res.data_ptr(),
                              d_risk.data_ptr())
    torch.cuda.synchronize()
    assert torch.all(d_risk == 0)
