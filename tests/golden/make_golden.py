"""Write the oracle's expected per-scenario records for the parity tests.

Calls only the oracle (and the shared input generators).  Outputs
tests/golden/<case>_oracle.npz with the outage list, the oracle's records,
island labels and the Risk Index over that list.

  c1_30:  every N-1 and N-2 branch outage of the 30-bus case (861 scenarios)
  c2_118: every N-1 outage plus a seeded sample of N-2 outages of the
          118-bus-shaped case (a stratified sample; the full list has 57,630)
  c2_118_full: the whole 57,630-scenario list of the 118-bus-shaped case

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
SAMPLES = {"c1_30": None, "c2_118": 600, "c2_118_full": None}
CASE_OF = {"c2_118_full": "c2_118"}
_NET = None


def _init(path):
    global _NET
    warnings.simplefilter("ignore")
    _NET = netgen.load_case(path)


def _one(o):
    r = screen.evaluate(_NET, o, detail=True)
    return r


def case_list(net, name):
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
    out = os.path.join(HERE, name + "_oracle.npz")
    np.savez_compressed(out, outages=lst, labels=labels, risk=R, **tab)
    print(f"{name}: {len(lst)} scenarios, {int(tab['severe'].sum())} severe -> {out}")


if __name__ == "__main__":
    procs = int(os.environ.get("GOLDEN_PROCS", "8"))
    for name in (sys.argv[1:] or ["c1_30", "c2_118"]):
        make(name, procs)
