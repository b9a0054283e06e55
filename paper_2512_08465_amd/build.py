"""Build the gfx950 screening library (libcs.so) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

COMPILE_TIMEOUT_S = 900
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcs.so")
SOURCES = ["k_topology.hip", "k_opf.hip", "k_dense.hip", "k_mixed.hip", "k_dyn.hip",
           "k_eig.hip", "k_finalize.hip", "k_risk.hip", "k_prune.hip", "k_lu_big.hip", "cs_abi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall", "-pthread",
         # loadable by the HIP runtime that PyTorch ships (one runtime per process)
         "-mcode-object-version=5",
         "-Wno-unused-result",
         # packed FP32 instructions are kept out of every device build
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC, *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    ok = True
    for cmd, p in procs:
        try:
            out, _ = p.communicate(timeout=COMPILE_TIMEOUT_S)
        except subprocess.TimeoutExpired:
            p.kill()
            out, _ = p.communicate()
            out += f"\ncompilation exceeded {COMPILE_TIMEOUT_S} s and was stopped\n"
        if p.returncode != 0 or verbose:
            sys.stderr.write(" ".join(cmd) + "\n" + out)
        ok &= p.returncode == 0
    if not ok:
        raise RuntimeError("hipcc compilation failed")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-mcode-object-version=5", "-shared", "-fPIC",
           "-pthread", *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
