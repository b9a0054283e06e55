"""Throughput of the per-contingency screening loop on one MI355X.

Workload: the 118-bus-shaped synthetic network (186 branches, 54 synchronous
generators, 99 loads) with every N-1 and unordered N-2 outage of its 339
components (57,630 scenarios).  The timed steps screen that list exactly once
(step k takes the k-th of K consecutive slices) through the whole path
(islanding, OPF with dense KKT LU, state matrix, eigenvalues, severity, Risk
Index) with the outage list, failure rates and outputs resident in device
memory: first in FP64 (the headline), then in the mixed-precision form
(FP32 KKT factorisation with FP64 refinement).  Then a serving sweep over
arrival rates in both precisions.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs fp64,mixed]
                  [--no-cpu-baseline] [--serve-requests R] [--serve-rates 2,20,200]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The host-side oracle baseline runs one BLAS thread in each of its (at most
# 16) worker processes; set before NumPy loads so no BLAS thread pool exists
# when the workers are forked.
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

METRIC = "N-2 scenarios/s (OPF+eigs) on 118-bus shape; p99 request latency; FP64 vs mixed"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3


def kkt_lu_flops(n: int) -> float:
    """Dense LU with partial pivoting (2/3 n^3) plus one forward and one back
    substitution (2 n^2) of an order-n system."""
    return 2.0 / 3.0 * n ** 3 + 2.0 * n ** 2


def cpu_baseline(case, lst, n_sample=512, seed=7):
    """The oracle timed on this host's cores on a seeded sample of the list.

    Runs before the device is initialised; workers are forked from this
    process, so they share its loaded modules and the network."""
    import numpy as np
    from multiprocessing import get_context
    from oracle import screen  # noqa: F401  (warm import before the fork)
    global _CPU_NET
    _CPU_NET = case
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(lst), n_sample, replace=False))
    cores = min(len(os.sched_getaffinity(0)), 16)
    ctx = get_context("fork")
    t0 = time.perf_counter()
    done = 0
    with ctx.Pool(cores) as p:
        for _ in p.imap_unordered(_cpu_one, [tuple(int(v) for v in lst[i]) for i in idx]):
            done += 1
            if done % 16 == 0:
                log(f"oracle: {done}/{n_sample} scenarios, {time.perf_counter() - t0:.1f} s")
    dt = time.perf_counter() - t0
    return dict(value=round(n_sample / dt, 3), unit="scenarios/s", cores=cores, kind="oracle",
                nproc=os.cpu_count(), affinity=len(os.sched_getaffinity(0)),
                cpu_model=cpu_model(),
                sample=f"{n_sample} scenarios drawn uniformly (seed {seed}) from the 57,630-row "
                       f"list, {cores} forked single-threaded worker processes (the host's "
                       f"share of cores, at most 16), {dt:.1f} s wall")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


_CPU_NET = None


def _cpu_one(o):
    import warnings
    warnings.simplefilter("ignore")
    from oracle import screen
    return screen.evaluate(_CPU_NET, o).severe


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4,
                    help="timed steps; together they screen the whole list exactly once")
    ap.add_argument("--warmup", type=int, default=1,
                    help="untimed steps, each over the first --warmup-size scenarios")
    ap.add_argument("--warmup-size", type=int, default=4096)
    ap.add_argument("--batch", type=int, default=8192,
                    help="scenario slots resident at once (refilled as scenarios finish)")
    ap.add_argument("--legs", default="fp64,mixed",
                    help="precisions to time: fp64 (the headline) and/or mixed")
    ap.add_argument("--graph", type=int, default=0,
                    help="Newton steps replayed from a captured HIP graph per round (0: eager)")
    ap.add_argument("--overlap", type=int, default=0,
                    help="1: dynamic stage on a second stream beside the OPF iterations; "
                         "2: the same, started only in the OPF tail at the end of a list")
    ap.add_argument("--c3-slice", type=int, default=14408,
                    help="scenarios of the converter case (c3_118) screened in FP64 and "
                         "mixed after the headline legs (0: skip)")
    ap.add_argument("--c4-slice", type=int, default=512,
                    help="scenarios of the 300-bus-shaped case (random branch/generator "
                         "pairs) screened in the mixed form and in FP64 (0: skip)")
    ap.add_argument("--c4-panel", type=int, default=0,
                    help="launch variant of the large-order LU (16, 32, 64, 1664, 3264); 0 = autotuned")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=12,
                    help="requests per arrival rate in the serving sweep (0: skip it)")
    ap.add_argument("--serve-rates", default="2,20,200", help="Poisson arrivals per second")
    ap.add_argument("--serve-max-len", type=int, default=5000,
                    help="request lengths are log-uniform integers in [1, this]")
    ap.add_argument("--serve-legs", default="fp64,mixed")
    ap.add_argument("--serve-mixed-sizes", type=int, default=1,
                    help="1: also serve 118- and 300-bus requests from one server")
    ap.add_argument("--pmc-copy", action="store_true",
                    help="begin with a device copy of known size (the scale of the HBM "
                         "counters in a counter pass over this run)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run only a copy of known size and a batch of order-580 LUs "
                         "(for hardware-counter passes), then exit")
    args = ap.parse_args()
    if args.pmc_probe:
        pmc_probe()
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(scenarios shard trivially across GPUs, but only the single-GPU path exists)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from inputs import netgen, contingencies

    case = netgen.load_case(os.path.join(ROOT, "inputs", "cases", "c2_118.npz"))
    lst = contingencies.n1_n2(case["outage_set"]).astype(np.int32)
    n_all = len(lst)
    step = -(-n_all // args.steps)
    legs = [v for v in args.legs.split(",") if v]
    assert legs and legs[0] == "fp64" or legs == ["mixed"], "--legs: fp64 first"
    base = None
    if not args.no_cpu_baseline:
        # before any device initialisation: worker processes are started here
        log("timing the oracle on the host cores")
        base = cpu_baseline(case, lst)
        log(f"oracle: {base['value']} scenarios/s on {base['cores']} cores")

    log("importing torch and the library")
    import torch
    import paper_2512_08465_amd as cs

    ctx = cs.Context(0)
    log("device context ready")
    if args.pmc_copy:
        src = torch.ones(PMC_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"pmc copy of {PMC_COPY_BYTES} bytes done")
    net = cs.Network(ctx, case)
    log(f"network resident; {n_all} scenarios, {step} per timed step")
    dev = torch.device("cuda:0")
    d_list = torch.from_numpy(lst).to(dev)
    d_lam = torch.from_numpy(case["lam"]).to(dev)
    d_res = torch.zeros(n_all * cs.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    d_risk = torch.zeros(len(case["lam"]), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    rec = cs.RESULT_DTYPE.itemsize
    golden = load_oracle_records()

    def run(off, cnt, opts):
        net.screen_device(d_list.data_ptr() + off * 8, cnt, d_lam.data_ptr(),
                          d_res.data_ptr() + off * rec, d_risk.data_ptr(), opts,
                          stream=stream.cuda_stream)
        return cnt

    results = {}
    for leg in legs:
        prec = cs.PREC_MIXED if leg == "mixed" else cs.PREC_FP64
        plain = cs.default_options(batch=args.batch, overlap=args.overlap, prec=prec,
                                   graph=args.graph)
        # (kernel timing launches every kernel itself: the timed steps run
        # eagerly, with the graph only when --graph is given and timing off)
        timed = cs.default_options(batch=args.batch, overlap=args.overlap, prec=prec,
                                   timing=0 if args.graph else 1, graph=args.graph)
        for w in range(args.warmup):
            run(0, min(args.warmup_size, n_all), plain)
            log(f"{leg}: warmup step {w + 1}/{args.warmup} done")
        torch.cuda.synchronize()
        ctx.reset_stats()
        done = 0
        t0 = time.perf_counter()
        for k in range(args.steps):
            off = k * step
            done += run(off, min(step, n_all - off), timed)
            log(f"{leg}: timed step {k + 1}/{args.steps} done ({done} scenarios)")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = d_res.cpu().numpy().view(cs.RESULT_DTYPE).copy()
        results[leg] = leg_summary(leg, ctx.stats(), done, dt, args.steps, res, golden)
        log(f"{leg}: {results[leg]['value']} scenarios/s")

    head = results[legs[0]]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "scenarios/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if legs[0] == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "c2_118: seeded synthetic 118-bus-shaped network (186 branches, "
                        "54 synchronous generators with AVR and governor, 99 loads); "
                        "N-1 + unordered N-2 over all 339 components = 57,630 scenarios, "
                        "screened once across the timed steps; " +
                        ("FP64 plain method" if legs[0] == "fp64" else
                         "KKT LU in FP32 with FP64 refinement, everything else FP64"),
            "scenarios_per_step": step,
            "slots": args.batch,
            "overlap": args.overlap,
            "graph_steps": args.graph,
            "kkt_order": head["kkt_order"],
            "state_order": 7 * int(case["n_gen"]) - 1,
        },
        "roofline": head.pop("roofline"),
        "kernel_time_share": head.pop("kernel_time_share"),
        "kkt_solves": head.pop("kkt_solves"),
        "results": head.pop("results"),
        "vs_oracle": head.pop("vs_oracle"),
    }
    if "mixed" in results and legs[0] == "fp64":
        out["mixed"] = results["mixed"]
    if args.c3_slice > 0:
        out["c3"] = c3_legs(cs, ctx, torch, args, lst)
    if args.c4_slice > 0:
        out["c4"] = c4_legs(cs, ctx, torch, args)
    if args.serve_requests > 0:
        out["serving"] = serve_sweep(cs, ctx, net, case, lst, args)
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


def c3_legs(cs, ctx, torch, args, lst):
    """The converter case (16 of the 54 machines replaced by grid-following
    converters, 393 states): the first c3_slice scenarios of the same list,
    FP64 and mixed, with the largest deviation of the mixed records from the
    FP64 ones."""
    import numpy as np
    from inputs import netgen
    case = netgen.load_case(os.path.join(ROOT, "inputs", "cases", "c3_118.npz"))
    net = cs.Network(ctx, case)
    n = min(args.c3_slice, len(lst))
    dev = torch.device("cuda:0")
    d_list = torch.from_numpy(np.ascontiguousarray(lst[:n])).to(dev)
    d_lam = torch.from_numpy(case["lam"]).to(dev)
    rec = cs.RESULT_DTYPE.itemsize
    out, recs = {"scenarios": n, "state_order": net.n_states_max}, {}
    for leg in ("fp64", "mixed"):
        prec = cs.PREC_MIXED if leg == "mixed" else cs.PREC_FP64
        d_res = torch.zeros(n * rec, dtype=torch.uint8, device=dev)
        d_risk = torch.zeros(len(case["lam"]), dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        net.screen_device(d_list.data_ptr(), min(n, args.warmup_size), d_lam.data_ptr(),
                          d_res.data_ptr(), d_risk.data_ptr(),
                          cs.default_options(batch=args.batch, prec=prec), stream=stream)
        torch.cuda.synchronize()
        ctx.reset_stats()
        t0 = time.perf_counter()
        net.screen_device(d_list.data_ptr(), n, d_lam.data_ptr(), d_res.data_ptr(),
                          d_risk.data_ptr(), cs.default_options(batch=args.batch, prec=prec,
                                                                timing=1), stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.stats()
        lu = st["kkt_lu"]
        nk = int(st["kkt_order"])
        per = lu["units"] / max(lu["launches"], 1)
        avg = lu["ms"] / max(lu["launches"], 1)
        ach = per * kkt_lu_flops(nk) / (avg * 1e-3) / 1e12 if lu["ms"] else 0.0
        peak = PEAK_FP32_TFLOPS if leg == "mixed" else PEAK_FP64_TFLOPS
        total_ms = sum(v["ms"] for v in st.values() if isinstance(v, dict))
        out[leg] = {"value": round(n / dt, 3), "unit": "scenarios/s",
                    "kkt_lu_tflops": round(ach, 4), "kkt_lu_frac": round(ach / peak, 5),
                    "kernel_time_share": {k: round(v["ms"] / max(total_ms, 1e-9), 4)
                                          for k, v in st.items()
                                          if isinstance(v, dict) and v["ms"] > 0},
                    "eig_share": round(st["eig"]["ms"] / max(sum(
                        v["ms"] for v in st.values() if isinstance(v, dict)), 1e-9), 4)}
        if leg == "mixed":
            # of the KKT factorisations, those in FP64 (a failed refinement's
            # fallback, or a scenario that stays on FP64 after one)
            out[leg]["fp64_factorisation_share"] = round(
                st["kkt_lu64"]["units"] / max(lu["units"] + st["kkt_lu64"]["units"], 1), 4)
        recs[leg] = d_res.cpu().numpy().view(cs.RESULT_DTYPE).copy()
        log(f"c3 {leg}: {out[leg]['value']} scenarios/s")
    a, b = recs["fp64"], recs["mixed"]
    both = (a["opf_status"] == 0) & (b["opf_status"] == 0)
    out["mixed_vs_fp64"] = {
        "severity_differs": int((a["severe"] != b["severe"]).sum()),
        "opf_cost_rel": float(np.max(np.abs(a["opf_cost"][both] - b["opf_cost"][both])
                                     / np.abs(a["opf_cost"][both]))),
        "max_real_eig": float(np.max(np.abs(a["max_real_eig"][both] - b["max_real_eig"][both])
                                     / np.maximum(np.abs(a["max_real_eig"][both]), 1.0))),
        "min_damping": float(np.max(np.abs(a["min_damping"][both] - b["min_damping"][both])))}
    net.close()
    return out


def c4_legs(cs, ctx, torch, args):
    """The 300-bus-shaped case (411 branches, 69 machines, 200 loads; KKT
    order 1,338, 482 states): the head of its list of random branch/generator
    pairs in the mixed form (FP32 KKT factorisation with FP64 refinement, the
    form this workload is specified in) and in FP64."""
    import numpy as np
    from inputs import netgen, contingencies
    case = netgen.load_case(os.path.join(ROOT, "inputs", "cases", "c4_300.npz"))
    lst = contingencies.c4_list(case["outage_set"])
    net = cs.Network(ctx, case)
    n = min(args.c4_slice, len(lst))
    dev = torch.device("cuda:0")
    d_list = torch.from_numpy(np.ascontiguousarray(lst[:n])).to(dev)
    d_lam = torch.from_numpy(case["lam"]).to(dev)
    rec = cs.RESULT_DTYPE.itemsize
    nk = 4 * int(case["n_bus"]) + 2 * int(case["n_gen"])
    out = {"scenarios": n, "list": "20,000 seeded random branch/generator pairs",
           "kkt_order": nk, "state_order": net.n_states_max}
    # the large-order LU's panel width, tuned for this order and slot count
    # before the timed legs (cs_autotune)
    tune = {}
    for leg, prec in (("fp64", cs.PREC_FP64), ("mixed", cs.PREC_MIXED)):
        if args.c4_panel:
            ctx.autotune_set(nk, prec, args.c4_panel)
            tune[leg] = {"variant": args.c4_panel, "variants": list(cs.TUNE_VARIANTS), "ms": None}
            continue
        choice, ms = ctx.autotune(nk, prec, n)
        tune[leg] = {"variant": choice, "variants": list(cs.TUNE_VARIANTS),
                     "ms": [round(float(v), 2) for v in ms]}
    out["autotune"] = tune
    for leg in ("mixed", "fp64"):
        prec = cs.PREC_MIXED if leg == "mixed" else cs.PREC_FP64
        d_res = torch.zeros(n * rec, dtype=torch.uint8, device=dev)
        d_risk = torch.zeros(len(case["lam"]), dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        ctx.reset_stats()
        t0 = time.perf_counter()
        net.screen_device(d_list.data_ptr(), n, d_lam.data_ptr(), d_res.data_ptr(),
                          d_risk.data_ptr(), cs.default_options(prec=prec, timing=1),
                          stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.stats()
        lu = st["kkt_lu"]
        nk = int(st["kkt_order"])
        per = lu["units"] / max(lu["launches"], 1)
        avg = lu["ms"] / max(lu["launches"], 1)
        ach = per * kkt_lu_flops(nk) / (avg * 1e-3) / 1e12 if lu["ms"] else 0.0
        peak = PEAK_FP32_TFLOPS if leg == "mixed" else PEAK_FP64_TFLOPS
        res = d_res.cpu().numpy().view(cs.RESULT_DTYPE)
        total_ms = sum(v["ms"] for v in st.values() if isinstance(v, dict))
        out[leg] = {"value": round(n / dt, 3), "unit": "scenarios/s",
                    "kkt_lu_tflops": round(ach, 4), "kkt_lu_frac": round(ach / peak, 5),
                    "kernel_time_share": {k: round(v["ms"] / max(total_ms, 1e-9), 4)
                                          for k, v in st.items()
                                          if isinstance(v, dict) and v["ms"] > 0},
                    "islanded_fraction": round(float(np.mean(res["n_islands"] > 1)), 4),
                    "severe_fraction": round(float(np.mean(res["severe"])), 4)}
        if leg == "mixed":
            # of the KKT factorisations, those in FP64 (a failed refinement's
            # fallback, or a scenario that stays on FP64 after one)
            out[leg]["fp64_factorisation_share"] = round(
                st["kkt_lu64"]["units"] / max(lu["units"] + st["kkt_lu64"]["units"], 1), 4)
        log(f"c4 {leg}: {out[leg]['value']} scenarios/s")
    net.close()
    return out


def load_oracle_records():
    """The oracle's stored records of the whole list (tests/golden), for the
    deviation figures; None if absent."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "c2_118_full_oracle.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in ("severe", "opf_status", "opf_cost", "max_real_eig",
                                  "min_damping", "n_islands")}


def leg_summary(leg, st, done, dt, steps, res, golden):
    import numpy as np
    mixed = leg == "mixed"
    nk = int(st["kkt_order"])
    lu = st["kkt_lu"]
    lu_avg_ms = lu["ms"] / max(lu["launches"], 1)
    per_launch = lu["units"] / max(lu["launches"], 1)
    achieved = per_launch * kkt_lu_flops(nk) / (lu_avg_ms * 1e-3) / 1e12 if lu["ms"] else 0.0
    peak = PEAK_FP32_TFLOPS if mixed else PEAK_FP64_TFLOPS
    lu_bytes = None if mixed else lu_traffic_per_factorisation()
    total_ms = sum(v["ms"] for v in st.values() if isinstance(v, dict))
    share = {k: round(v["ms"] / max(total_ms, 1e-9), 4) for k, v in st.items()
             if isinstance(v, dict)}
    status = res["opf_status"]
    iters = res["opf_iters"].astype(np.int64)
    out = {
        "value": round(done / dt, 3),
        "ms_per_step": round(1e3 * dt / steps, 3),
        "kkt_order": nk,
        "roofline": {
            # four wavefronts per matrix by default in FP64 (orders up to 768), eight
            # in FP32 and for FP64 launches with at most one system per compute unit
            "kernel": "k_lu_solve<%s, LU_KKT, %s> (KKT LU + solve)" % (
                ("float", "8") if mixed else ("double", "4 or 8" if nk <= 768 else "8")),
            "bound": "mfma",
            "achieved": round(achieved, 4),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 5),
            "traffic": None if lu_bytes is None else round(lu_bytes * per_launch / 1e9, 3),
            "traffic_unit": "GB per launch (HBM, counters)",
            "algorithmic_bytes_per_launch_gb": round(
                2 * (4 if mixed else 8) * nk * (nk + 1) * per_launch / 1e9, 3),
            "avg_launch_ms": round(lu_avg_ms, 4),
            "launches": int(lu["launches"]),
            "factorisations_per_launch": round(per_launch, 1),
        },
        "kernel_time_share": share,
        "kkt_solves": {"factorisations": int(lu["units"]),
                       "fp64_fallbacks": int(st["kkt_lu64"]["units"]) if mixed else None,
                       "fp64_factorisation_share": (
                           round(st["kkt_lu64"]["units"] /
                                 max(lu["units"] + st["kkt_lu64"]["units"], 1), 4)
                           if mixed else None)},
        "results": {
            "screened": int(done),
            "severe_fraction": round(float(np.mean(res["severe"])), 4),
            "opf_maxit_fraction": round(float(np.mean(status == 1)), 4),
            "opf_diverged_fraction": round(float(np.mean(status == 2)), 4),
            "newton_steps_at_maxit_share": round(float(iters[status == 1].sum() /
                                                       max(iters.sum(), 1)), 4),
            "newton_steps_histogram": np.histogram(iters[status != 3],
                                                   bins=[0, 20, 30, 40, 60, 100, 149, 151]
                                                   )[0].tolist(),
            "newton_steps_bins": [0, 20, 30, 40, 60, 100, 149, 151],
        },
        "vs_oracle": deviation(res, golden),
    }
    if mixed:
        out["dtype"] = "f32+f64"
    return out


def deviation(res, g):
    """Largest deviations of the screened records from the oracle's stored
    ones: on scenarios converged on both sides, OPF cost (relative), the
    largest real part (relative to max(|.|, 1)) and the minimum damping;
    and the number of scenarios whose severity differs."""
    import numpy as np
    if g is None:
        return None
    both = (g["opf_status"] == 0) & (res["opf_status"] == 0)
    rel = np.abs(res["opf_cost"][both] - g["opf_cost"][both]) / np.abs(g["opf_cost"][both])
    da = np.abs(res["max_real_eig"][both] - g["max_real_eig"][both]) / np.maximum(
        np.abs(g["max_real_eig"][both]), 1.0)
    dz = np.abs(res["min_damping"][both] - g["min_damping"][both])
    return {"converged_both": int(both.sum()),
            "opf_cost_rel": float(rel.max()), "max_real_eig": float(da.max()),
            "min_damping": float(dz.max()),
            "islands_differ": int((res["n_islands"] != g["n_islands"]).sum()),
            "severity_differs": int((res["severe"] != g["severe"]).sum())}


# HBM traffic of the FP64 KKT LU from two rocprofv3 counter passes over
# `python bench.py --steps 20 --warmup 0 --legs fp64 --no-cpu-baseline
# --serve-requests 0 --c3-slice 0 --c4-slice 0 --pmc-copy`
# (profiles/k_lu_solve_hbm_traffic_c2_118.md): FETCH_SIZE and WRITE_SIZE summed
# over the run's KKT LU dispatches (both launch geometries), each scaled by
# what the same counter reads for the run's 1 GiB device copy, divided by the
# factorisations those dispatches performed.  Valid only for the kernel source
# it was measured on (hash below); otherwise traffic is null.
LU_TRAFFIC = dict(source_sha256_16="3dae3a559862c5c6", factorisations=2217483,
                  fetch_kib=32023448784.25, write_kib=25146651497.5,
                  copy_fetch_kib=524307.8125, copy_write_kib=1048576.0,
                  copy_bytes=1 << 30)


def lu_traffic_per_factorisation():
    import hashlib
    src = os.path.join(ROOT, "paper_2512_08465_amd", "csrc", "k_dense.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != LU_TRAFFIC["source_sha256_16"]:
            return None
    t = LU_TRAFFIC
    kib = t["copy_bytes"] / 1024.0
    fetch = t["fetch_kib"] * kib / t["copy_fetch_kib"]
    write = t["write_kib"] * kib / t["copy_write_kib"]
    return (fetch + write) * 1024.0 / t["factorisations"]


PMC_COPY_BYTES = 1 << 30
PMC_LU_BATCH = 512
PMC_LU_ORDER = 580
PMC_EIG_BATCH = 1024
PMC_EIG_ORDER = 377


def pmc_probe():
    """Workloads for the FETCH_SIZE / WRITE_SIZE counter passes: a plain
    device copy of PMC_COPY_BYTES (the scale of the counters), then one batch
    of PMC_LU_BATCH random order-580 systems through the library's LU kernel
    (the KKT factorisation's kernel and shape), then one batch of
    PMC_EIG_BATCH random order-377 matrices through the eigenvalue kernel (the
    state matrices' order)."""
    import numpy as np
    import torch
    import paper_2512_08465_amd as cs
    ctx = cs.Context(0)
    src = torch.ones(PMC_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    n, k = PMC_LU_ORDER, 1
    lda = n + k + ((n + k) % 2)
    rng = np.random.default_rng(0)
    a = torch.from_numpy(rng.standard_normal((PMC_LU_BATCH, n, lda))).cuda()
    info = torch.zeros(PMC_LU_BATCH, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    ctx.dense_solve_batched(a.data_ptr(), n, k, lda, PMC_LU_BATCH, info.data_ptr())
    torch.cuda.synchronize()
    del a
    ne = PMC_EIG_ORDER
    h = torch.from_numpy(rng.standard_normal((PMC_EIG_BATCH, ne, ne))).cuda()
    wr = torch.zeros((PMC_EIG_BATCH, ne), dtype=torch.float64, device="cuda")
    wi = torch.zeros_like(wr)
    einfo = torch.zeros(PMC_EIG_BATCH, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    ctx.eigvals_batched(h.data_ptr(), ne, ne, PMC_EIG_BATCH, wr.data_ptr(), wi.data_ptr(),
                        einfo.data_ptr())
    torch.cuda.synchronize()
    log("pmc probe: copy, LU batch and eigenvalue batch done")


def serve_sweep(cs, ctx, net, case, lst, args):
    """Serving: for each precision and arrival rate, requests arriving as a
    Poisson process, each a random slice of the list with a log-uniform
    length, admitted into a running server; p50/p99 latency from admission
    to the last record and the scenarios served per second."""
    out = []
    for leg in [v for v in args.serve_legs.split(",") if v]:
        prec = cs.PREC_MIXED if leg == "mixed" else cs.PREC_FP64
        for rate in [float(v) for v in args.serve_rates.split(",") if v]:
            r = serve(cs, ctx, net, case, lst, args, rate, prec)
            r["prec"] = leg
            out.append(r)
            log(f"serving {leg} at {rate}/s: p50 {r['p50_latency_s']} s, "
                f"p99 {r['p99_latency_s']} s, {r['scenarios_per_s']} scenarios/s")
    if args.serve_mixed_sizes:
        r = serve_two_sizes(cs, ctx, net, case, lst, args)
        out.append(r)
        log(f"serving 118- and 300-bus requests: p99 {r['p99_latency_s']} s, "
            f"{r['scenarios_per_s']} scenarios/s")
    return out


def serve_two_sizes(cs, ctx, net, case, lst, args):
    """One server for the 118- and the 300-bus networks under one HBM
    budget (cs_server_create_multi): 12 requests at 20 per second, every
    fourth a 300-bus snapshot with 1-200 random pairs of its list, the others
    118-bus snapshots with 1-5,000 scenarios; p50/p99 latency per network."""
    import numpy as np
    from inputs import netgen, contingencies
    from inputs.rate_samples import load_scales
    c4 = netgen.load_case(os.path.join(ROOT, "inputs", "cases", "c4_300.npz"))
    lst4 = contingencies.c4_list(c4["outage_set"])
    net4 = cs.Network(ctx, c4)
    rng = np.random.default_rng(7300)
    nreq, rate = 12, 20.0
    gaps = rng.exponential(1.0 / rate, nreq)
    kinds = [1 if i % 4 == 3 else 0 for i in range(nreq)]
    reqs_in = []
    for i, k in enumerate(kinds):
        top = 200 if k else args.serve_max_len
        m = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(top + 1)))), 1, top))
        src, cc = (lst4, c4) if k else (lst, case)
        sc = load_scales(int(cc["n_load"]), 1, seed=7300 + i)[0]
        reqs_in.append((k, src[rng.choice(len(src), m, replace=False)], cc, sc))
    budget = 48 << 30
    srv = cs.Server(ctx, [net, net4], cs.default_options(hbm_budget=budget, batch=4096),
                    queue_capacity=1 << 16, shares=[1.0, 1.0])
    slots = [srv.slots(0), srv.slots(1)]
    t0 = time.perf_counter()
    due = t0
    reqs = []
    for g, (k, l, cc, sc) in zip(gaps, reqs_in):
        due += g
        time.sleep(max(0.0, due - time.perf_counter()))
        reqs.append((k, len(l), srv.submit(l, cc["lam"], load_scale=sc, net=k)))
    lat = {0: [], 1: []}
    for k, m, r in reqs:
        _, _, t = r.wait(timeout_s=900)
        lat[k].append(t)
        r.close()
    dt = time.perf_counter() - t0
    srv.close()
    net4.close()
    total = sum(m for _, m, _ in reqs)
    allat = np.array(lat[0] + lat[1])
    return dict(requests=nreq, rate_per_s=rate, networks="118-bus and 300-bus in one server",
                hbm_budget_gib=budget >> 30, slots_118_300=slots,
                length="118-bus: log-uniform [1, %d]; 300-bus: log-uniform [1, 200]"
                % args.serve_max_len,
                scenarios=int(total), prec="fp64",
                p50_latency_s=round(float(np.percentile(allat, 50)), 4),
                p99_latency_s=round(float(np.percentile(allat, 99)), 4),
                p99_latency_118_s=round(float(np.percentile(lat[0], 99)), 4),
                p99_latency_300_s=round(float(np.percentile(lat[1], 99)), 4),
                scenarios_per_s=round(total / dt, 2), wall_s=round(dt, 2))


def serve(cs, ctx, net, case, lst, args, rate, prec):
    import numpy as np
    rng = np.random.default_rng(5000 + int(rate * 10))
    nreq = args.serve_requests
    gaps = rng.exponential(1.0 / rate, nreq)
    lens = np.floor(np.exp(rng.uniform(0, np.log(args.serve_max_len + 1), nreq)))
    lens = np.clip(lens.astype(int), 1, args.serve_max_len)
    lists = [lst[rng.choice(len(lst), k, replace=False)] for k in lens]
    # each request screens its own snapshot: every load times N(1, 0.05)
    from inputs.rate_samples import load_scales
    scales = load_scales(int(case["n_load"]), nreq, seed=5000 + int(rate * 10))
    slots = 4096
    srv = cs.Server(ctx, net, cs.default_options(batch=slots, prec=prec),
                    queue_capacity=1 << 17)
    reqs = []
    t0 = time.perf_counter()
    due = t0
    for g, l, sc in zip(gaps, lists, scales):
        due += g
        time.sleep(max(0.0, due - time.perf_counter()))
        reqs.append(srv.submit(l, case["lam"], load_scale=sc))
    lat = []
    for r in reqs:
        _, _, l = r.wait(timeout_s=600)
        lat.append(l)
        r.close()
    dt = time.perf_counter() - t0
    srv.close()
    lat = np.array(lat)
    return dict(requests=int(nreq), rate_per_s=rate,
                length="log-uniform integer in [1, %d]" % args.serve_max_len,
                snapshot="every load of a request times N(1, 0.05)",
                scenarios=int(lens.sum()), slots=slots,
                p50_latency_s=round(float(np.percentile(lat, 50)), 4),
                p99_latency_s=round(float(np.percentile(lat, 99)), 4),
                scenarios_per_s=round(float(lens.sum()) / dt, 2),
                wall_s=round(dt, 2))


if __name__ == "__main__":
    main()
