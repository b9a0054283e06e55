"""Launch-shape machinery through the C-ABI: the Newton step replayed from a
captured HIP graph (opts.graph) and the large-order LU's panel widths with
the autotuner that chooses among them (cs_autotune, opts.autotune).

* Graph replays: every scheduling round replays the captured Newton step k
  times between the engine's own eager kernels (refill, stage counts, the
  dynamic stage) and host synchronisations; the records and R_i of a whole
  list are bit-identical to the eager launches', FP64 and mixed, in a batch
  call and in a server.
* Every launch variant of the large-order LU (panel widths 16, 32 and 64,
  and panels of 16 or 32 in groups of 64) gives factors and solutions equal
  to SciPy's (LAPACK's pivoting) at orders 1,100 and 1,338; the autotuner
  returns the fastest of its own timings.
* The register-resident LU at four and at eight wavefronts per matrix gives
  the same bits (factors, pivots' effect, solutions) at orders that span one,
  two and three panel rows per thread, and the same screening records, FP64
  and mixed; the autotuner picks between the two up to order 768 and keeps
  eight above.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from helpers import load_case, load_golden

pytestmark = pytest.mark.gpu

FIELDS = ("severe", "cause", "opf_status", "near", "n_islands", "opf_iters", "n_states",
          "opf_cost", "max_real_eig", "min_damping", "max_violation")


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_08465_amd as cs
    return cs.Context(0)


@pytest.fixture(scope="module")
def nets(ctx):
    import paper_2512_08465_amd as cs
    return {k: (cs.Network(ctx, load_case(k)), load_case(k)) for k in ("c1_30", "c2_118")}


def _same(a, b):
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), \
        [k for k in FIELDS if not np.array_equal(a[k], b[k], equal_nan=True)]


@pytest.mark.parametrize("prec,steps", [(0, 1), (0, 3), (1, 2)])
def test_graph_replays_equal_eager_c1(nets, prec, steps):
    import paper_2512_08465_amd as cs
    net, case = nets["c1_30"]
    lst = load_golden("c1_30")["outages"]
    print(f"c1_30: {len(lst)} scenarios, prec {prec}, {steps} replays per round", flush=True)
    ref, ref_r = net.screen(lst, case["lam"], cs.default_options(prec=prec, batch=200))
    got, got_r = net.screen(lst, case["lam"], cs.default_options(prec=prec, batch=200, graph=steps))
    _same(got, ref)
    assert np.array_equal(got_r, ref_r)


def test_graph_replays_equal_eager_c2(nets):
    import paper_2512_08465_amd as cs
    net, case = nets["c2_118"]
    lst = load_golden("c2_118")["outages"][:300]
    print(f"c2_118: {len(lst)} scenarios", flush=True)
    ref, ref_r = net.screen(lst, case["lam"], cs.default_options(batch=128))
    got, got_r = net.screen(lst, case["lam"], cs.default_options(batch=128, graph=1))
    _same(got, ref)
    assert np.array_equal(got_r, ref_r)


def test_graph_in_a_server(nets):
    import paper_2512_08465_amd as cs
    net, case = nets["c1_30"]
    g = load_golden("c1_30")["outages"]
    lists = [g[:150], g[400:470], g[700:861]]
    srv = cs.Server(net.ctx, net, cs.default_options(batch=64, graph=2), queue_capacity=2048)
    reqs = [srv.submit(l, case["lam"]) for l in lists]
    for l, r in zip(lists, reqs):
        res, risk, _ = r.wait(timeout_s=300)
        ref, ref_r = net.screen(l, case["lam"])
        _same(res, ref)
        assert np.array_equal(risk, ref_r)
    srv.close()


def test_noalloc_refuses_graph_and_autotune(nets):
    import torch
    import paper_2512_08465_amd as cs
    net, case = nets["c1_30"]
    d_rows = torch.tensor([[0, -1]], dtype=torch.int32, device="cuda")
    d_out = torch.zeros(cs.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    for kw in (dict(graph=1), dict(autotune=1)):
        with pytest.raises(cs.CSError) as e:
            net.screen_device_noalloc(d_rows.data_ptr(), 1, None, d_out.data_ptr(), None,
                                      cs.default_options(**kw))
        assert e.value.code == cs.CS_EINVAL


def _run_lu(ctx, A, rhs):
    import torch
    B, n, _ = A.shape
    k = rhs.shape[2]
    lda = n + k + ((n + k) % 2)
    buf = np.zeros((B, n, lda))
    buf[:, :, :n] = A
    buf[:, :, n:n + k] = rhs
    d = torch.from_numpy(buf).cuda()
    info = torch.zeros(B, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    ctx.dense_solve_batched(d.data_ptr(), n, k, lda, B, info.data_ptr())
    out = d.cpu().numpy()
    return out[:, :, :n], out[:, :, n:], info.cpu().numpy()


@pytest.mark.parametrize("n", [1100, 1338])
@pytest.mark.parametrize("nb", [16, 32, 64, 1664, 3264])
def test_panel_widths_match_scipy(ctx, n, nb):
    rng = np.random.default_rng(n + nb)
    A = rng.standard_normal((2, n, n))
    X = rng.standard_normal((2, n, 2))
    ctx.autotune_set(n, 0, nb)
    try:
        fac, sol, info = _run_lu(ctx, A, A @ X)
    finally:
        ctx.autotune_set(n, 0, 0)
    assert np.all(info == 0)
    for b in range(2):
        lu, piv = sla.lu_factor(A[b])
        assert np.allclose(fac[b], lu, rtol=1e-9, atol=1e-9 * np.abs(lu).max())
        ref = sla.lu_solve((lu, piv), (A @ X)[b])
        assert np.max(np.abs(sol[b] - ref)) <= 1e-13 * np.linalg.cond(A[b]) * max(1, np.abs(ref).max())


def test_autotune_picks_its_fastest(ctx):
    import paper_2512_08465_amd as cs
    choice, ms = ctx.autotune(1338, cs.PREC_FP64, 256)
    print(f"order 1338 FP64: variants {cs.TUNE_VARIANTS} take {ms} ms; chose {choice}")
    assert choice in cs.TUNE_VARIANTS
    assert np.all(np.isfinite(ms)) and np.all(ms > 0)
    assert choice == cs.TUNE_VARIANTS[int(np.argmin(ms))]
    choice32, ms32 = ctx.autotune(1338, cs.PREC_MIXED, 256)
    print(f"order 1338 FP32: {ms32} ms; chose {choice32}")
    assert choice32 == cs.TUNE_VARIANTS[int(np.argmin(ms32))]
    ctx.autotune_set(1338, cs.PREC_FP64, 0)
    ctx.autotune_set(1338, cs.PREC_MIXED, 0)
    with pytest.raises(cs.CSError) as e:
        ctx.autotune_set(1338, cs.PREC_FP64, 48)
    assert e.value.code == cs.CS_EINVAL


def test_autotuned_c4_records_match_oracle(ctx):
    """opts.autotune on the 300-bus case (KKT order 1,338): the tuned run's
    records agree with the oracle's to the usual bars, FP64 and mixed."""
    import paper_2512_08465_amd as cs
    from helpers import outcome_mismatches
    case = load_case("c4_300")
    net = cs.Network(ctx, case)
    g = load_golden("c4_300")
    idx = np.flatnonzero(g["opf_iters"] < 40)[:12]
    for prec in (cs.PREC_FP64, cs.PREC_MIXED):
        res, _ = net.screen(g["outages"][idx], None, cs.default_options(prec=prec, autotune=1))
        sub = {k: g[k][idx] for k in g if len(g[k]) == len(g["outages"])}
        bad, _, _ = outcome_mismatches(sub, res)
        assert len(bad) == 0, bad
        both = (sub["opf_status"] == 0) & (res["opf_status"] == 0)
        rel = np.abs(res["opf_cost"][both] - sub["opf_cost"][both]) / np.abs(sub["opf_cost"][both])
        assert rel.max() < 1e-6
    net.close()
    ctx.autotune_set(1338, cs.PREC_FP64, 0)
    ctx.autotune_set(1338, cs.PREC_MIXED, 0)


@pytest.mark.parametrize("n,k", [(1, 1), (33, 2), (200, 3), (344, 162), (513, 1), (580, 1),
                                 (768, 2)])
def test_wave_counts_give_the_same_bits(ctx, n, k):
    """Four and eight wavefronts per matrix run the same operations on every
    element: factors and solutions are equal bit for bit (and equal SciPy's
    to rounding)."""
    rng = np.random.default_rng(7 * n + k)
    A = rng.standard_normal((3, n, n))
    rhs = A @ rng.standard_normal((3, n, k))
    out = {}
    try:
        for w in (8, 4):
            ctx.autotune_set(n, 0, w)
            out[w] = _run_lu(ctx, A, rhs)
    finally:
        ctx.autotune_set(n, 0, 0)
    for a, b in zip(out[8], out[4]):
        assert np.array_equal(a, b)
    fac, sol, info = out[4]
    assert np.all(info == 0)
    for b in range(3):
        lu, piv = sla.lu_factor(A[b])
        assert np.allclose(fac[b], lu, rtol=1e-9, atol=1e-9 * np.abs(lu).max())


def test_wave_counts_give_the_same_records(ctx):
    """A slice of the 118-bus-shaped list screened with the KKT LU (order 580)
    and the algebraic-system LU (order 344) at four and at eight wavefronts:
    identical records and R_i, FP64 and mixed (FP32 factorisation and FP64
    fallback)."""
    import paper_2512_08465_amd as cs
    case = load_case("c2_118")
    net = cs.Network(ctx, case)
    g = load_golden("c2_118")
    lst = g["outages"][:96]
    recs = {}
    try:
        for prec in (cs.PREC_FP64, cs.PREC_MIXED):
            for w in (8, 4):
                for order in (580, 344):
                    ctx.autotune_set(order, cs.PREC_FP64, w)
                    ctx.autotune_set(order, cs.PREC_MIXED, w)
                recs[prec, w] = net.screen(lst, case["lam"], cs.default_options(prec=prec))
    finally:
        for order in (580, 344):
            ctx.autotune_set(order, cs.PREC_FP64, 0)
            ctx.autotune_set(order, cs.PREC_MIXED, 0)
        net.close()
    for prec in (cs.PREC_FP64, cs.PREC_MIXED):
        (r8, R8), (r4, R4) = recs[prec, 8], recs[prec, 4]
        assert r8.tobytes() == r4.tobytes()
        assert np.array_equal(R8, R4)


def test_autotune_register_resident_orders(ctx):
    import paper_2512_08465_amd as cs
    try:
        for prec in (cs.PREC_FP64, cs.PREC_MIXED):
            choice, ms = ctx.autotune(580, prec, 512)
            print(f"order 580 prec {prec}: waves {cs.REG_TUNE_VARIANTS} take {ms[:2]} ms; "
                  f"chose {choice}")
            assert np.all(np.isfinite(ms[:2])) and np.all(ms[:2] > 0)
            assert np.all(np.isnan(ms[2:]))
            assert choice == cs.REG_TUNE_VARIANTS[int(np.argmin(ms[:2]))]
        # above order 768 only eight wavefronts fit
        choice, ms = ctx.autotune(900, cs.PREC_FP64, 64)
        assert choice == 8 and np.isnan(ms[0]) and np.isfinite(ms[1])
        with pytest.raises(cs.CSError) as e:
            ctx.autotune_set(900, cs.PREC_FP64, 4)
        assert e.value.code == cs.CS_EINVAL
        with pytest.raises(cs.CSError) as e:
            ctx.autotune_set(580, cs.PREC_FP64, 32)
        assert e.value.code == cs.CS_EINVAL
    finally:
        for n in (580, 900):
            ctx.autotune_set(n, cs.PREC_FP64, 0)
            ctx.autotune_set(n, cs.PREC_MIXED, 0)
