"""Write the oracle's expected per-scenario records for the parity tests.

Calls only the oracle (and the shared input generators).  Outputs
tests/golden/<case>_oracle.npz with the outage list, the oracle's records,
island labels and the Risk Index over that list.

  c1_30:  every N-1 and N-2 branch outage of the 30-bus case (861 scenarios)
  c2_118: every N-1 outage plus a seeded sample of N-2 outages of the
          118-bus-shaped case (a stratified sample; the full list has 57,630)
  c2_118_full: the whole 57,630-scenario list of the 118-bus-shaped case
  c3_118: the same stratified sample of the 118-bus shape with 16 machines
          replaced by grid-following converters (c3_118 case)
  c4_300: the first 200 of the 20,000 random branch/generator pairs of the
          300-bus-shaped case
  c1_30_n3: every N-3 triple of the 30-bus case's 41 branches (10,660 rows),
          all solved, with the pruning flags of screen.n3_prune (by c1_30's
          records) and R_i with pruned rows counted as severe

c1_30 and c2_118 also hold each scenario's operating point (vm, va over the
buses, pg, qg over the generators; NaN outside the solved island or when the
OPF did not run) and its full spectrum (eig_re, eig_im, NaN-padded, n_eig
values).

  python tests/golden/make_golden.py --refresh-near [case ...]

recomputes only the stored near-threshold flags from the stored records with
the oracle's own rule (oracle.screen.near_flags), without solving again.

Usage: python tests/golden/make_golden.py [case ...]
"""
from __future__ import annotations

import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import warnings                      # noqa: E402
from multiprocessing import Pool     # noqa: E402

import numpy as np                   # noqa: E402

from inputs import netgen, contingencies          # noqa: E402
from oracle import screen, risk                    # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLES = {"c1_30": None, "c2_118": 600, "c2_118_full": None, "c1_30_n3": None,
           "c3_118": 600, "c4_300": 200}
WITH_DETAIL = {"c1_30", "c2_118", "c3_118", "c4_300"}
CASE_OF = {"c2_118_full": "c2_118", "c1_30_n3": "c1_30"}
_NET = None


def _init(path):
    global _NET
    warnings.simplefilter("ignore")
    _NET = netgen.load_case(path)


def _one(o):
    r = screen.evaluate(_NET, o, detail=True)
    return r


def case_list(net, name):
    if name.endswith("_n3"):
        return contingencies.n3(net["outage_set"])
    if name == "c4_300":
        # the head of the 300-bus workload (random branch/generator pairs)
        return contingencies.c4_list(net["outage_set"])[:SAMPLES[name]]
    full = contingencies.n1_n2(net["outage_set"])
    n = SAMPLES[name]
    if n is None:
        return full
    return full[contingencies.stratified_sample(full, n, seed=2512)]


def make(name, procs=8):
    path = os.path.join(ROOT, "inputs", "cases", CASE_OF.get(name, name) + ".npz")
    net = netgen.load_case(path)
    lst = case_list(net, name)
    with Pool(procs, initializer=_init, initargs=(path,)) as p:
        res = []
        for k, r in enumerate(p.imap(_one, list(lst), chunksize=4)):
            res.append(r)
            if (k + 1) % 2000 == 0:
                print(f"{name}: {k + 1}/{len(lst)}", flush=True)
    tab = screen.as_table(res)
    labels = np.array([r.label for r in res], dtype=np.int16)
    n_comp = int(net["n_branch"]) + int(net["n_gen"]) + int(net["n_load"])
    R = risk.risk_index(lst, tab["severe"], net["lam"], n_comp)
    extra = detail_arrays(net, res) if name in WITH_DETAIL else {}
    if name.endswith("_n3"):
        # pruning by the oracle's own N-1/N-2 records of the same case; R_i
        # counts a pruned row as severe
        with np.load(os.path.join(HERE, CASE_OF[name] + "_oracle.npz"), allow_pickle=False) as z:
            keep = screen.n3_prune(lst, z["outages"], z["severe"])
        extra["keep"] = keep
        extra["risk_pruned"] = risk.risk_index(lst, tab["severe"] | ~keep, net["lam"], n_comp)
    out = os.path.join(HERE, name + "_oracle.npz")
    np.savez_compressed(out, outages=lst, labels=labels, risk=R, **tab, **extra)
    print(f"{name}: {len(lst)} scenarios, {int(tab['severe'].sum())} severe -> {out}")


def detail_arrays(net, res):
    nb, ng = int(net["n_bus"]), int(net["n_gen"])
    na = int(np.sum(np.where(net["gen_kind"] == 1, 8, 7))) - 1
    n = len(res)
    d = {k: np.full((n, nb), np.nan) for k in ("vm", "va")}
    d.update({k: np.full((n, ng), np.nan) for k in ("pg", "qg")})
    d.update({k: np.full((n, na), np.nan) for k in ("eig_re", "eig_im")})
    d["n_eig"] = np.zeros(n, np.int32)
    for i, r in enumerate(res):
        if r.vm is not None and r.opf_status != screen.opf.NOT_RUN:
            d["vm"][i, r.bus], d["va"][i, r.bus] = r.vm, r.va
            d["pg"][i, r.gen], d["qg"][i, r.gen] = r.pg, r.qg
        if r.eig is not None:
            d["eig_re"][i, :len(r.eig)] = r.eig.real
            d["eig_im"][i, :len(r.eig)] = r.eig.imag
            d["n_eig"][i] = len(r.eig)
    return d


def refresh_near(name):
    """Rewrite the stored near flags with the oracle's rule applied to the
    stored status, iteration count, limit excess and largest real part."""
    out = os.path.join(HERE, name + "_oracle.npz")
    with np.load(out, allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    g["near"] = np.array([screen.near_flags(int(s), int(it), float(v), float(a))
                          for s, it, v, a in zip(g["opf_status"], g["opf_iters"],
                                                 g["max_violation"], g["max_real_eig"])],
                         dtype=g["near"].dtype)
    np.savez_compressed(out, **g)
    print(f"{name}: near flags refreshed, {int((g['near'] > 0).sum())} flagged -> {out}")


if __name__ == "__main__":
    procs = int(os.environ.get("GOLDEN_PROCS", "8"))
    args = sys.argv[1:]
    if args and args[0] == "--refresh-near":
        for name in (args[1:] or ["c2_118_full"]):
            refresh_near(name)
        sys.exit(0)
    for name in (args or ["c1_30", "c2_118"]):
        make(name, procs)
