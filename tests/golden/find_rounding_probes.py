"""Find, for listed scenarios of the 118-bus-shaped list, a rounding probe
under which the oracle's own OPF outcome changes.

A probe solves every Newton system of the interior-point method by an exact
reformulation of the same step: Householder QR instead of LU, LU after
scaling the rows by powers of two, or LU of the system with its unknowns and
equations permuted.  In exact arithmetic none of them changes the iterates,
so an outcome that changes under one is decided by rounding, not by the
method (Section II.B.1 only asks whether the OPF converges).  Calls only the
oracle.

  python tests/golden/find_rounding_probes.py outcome ID[,ID...]
  python tests/golden/find_rounding_probes.py path ID[,ID...]
  python tests/golden/find_rounding_probes.py kind ID[,ID...]

outcome: a probe under which the OPF converges where the plain oracle's
does not, or the reverse.  path: the OPF converges under the probe too, but
its iteration count moves by more than two.  kind: both fail, one at the
iteration cap and one by divergence.  The first probe found (in the fixed
order below) is merged into tests/golden/c2_118_rounding_probes.json.
"""
from __future__ import annotations

import json
import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import warnings                      # noqa: E402
from multiprocessing import Pool     # noqa: E402

import numpy as np                   # noqa: E402

from inputs import netgen, contingencies          # noqa: E402
from oracle import screen                          # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "c2_118_rounding_probes.json")
PROBES = ([dict(kkt_solve="qr")] + [dict(row_scale_seed=k) for k in range(1, 41)]
          + [dict(perm_seed=k) for k in range(1, 41)])
_NET = None


def _init():
    global _NET
    warnings.simplefilter("ignore")
    _NET = netgen.load_case(os.path.join(ROOT, "inputs", "cases", "c2_118.npz"))


def _run(args):
    outage, probe = args
    r = screen.evaluate(_NET, np.array(outage), screen.ScreenOptions(**probe))
    return int(r.opf_status), int(r.opf_iters)


def changed(what, base, alt):
    (bs, bi), (s, i) = base, alt
    if what == "outcome":
        return (bs == 0) != (s == 0)
    if what == "path":
        return bs == 0 and s == 0 and abs(bi - i) > 2
    return bs not in (0, 3) and s not in (0, 3) and bs != s


def find(what, ids, procs=8):
    _init()
    lst = contingencies.n1_n2(_NET["outage_set"])
    found = {}
    with Pool(procs, initializer=_init) as p:
        for i in ids:
            outage = tuple(int(v) for v in lst[i])
            base = _run((outage, {}))
            for k in range(0, len(PROBES), procs):
                chunk = PROBES[k:k + procs]
                hits = [pr for pr, alt in zip(chunk, p.map(_run, [(outage, pr) for pr in chunk]))
                        if changed(what, base, alt)]
                if hits:
                    found[i] = dict(outage=list(outage), probe=hits[0])
                    break
            print(what, i, outage, "->", found.get(i, "no probe found"), flush=True)
    return found


if __name__ == "__main__":
    what, ids = sys.argv[1], [int(v) for v in sys.argv[2].split(",")]
    assert what in ("outcome", "path", "kind")
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    sect = data.setdefault(what, {})
    for i, v in find(what, ids).items():
        sect[str(i)] = v
    data[what] = dict(sorted(sect.items(), key=lambda kv: int(kv[0])))
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")
    print("->", OUT)
