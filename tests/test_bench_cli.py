"""The benchmark's command line on a host without the device: more than one
GPU is refused with a message and a non-zero status, before any device work,
and the traffic constants of the KKT LU are used only with the kernel source
they were measured on (else the benchmark reports the traffic as unknown)."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2",
                        "--no-cpu-baseline"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert '"metric"' not in r.stdout


def test_lu_traffic_constants_match_the_kernel_source():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    with open(os.path.join(ROOT, "paper_2512_08465_amd", "csrc", "k_dense.hip"), "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    per = b.lu_traffic_per_factorisation()
    if b.LU_TRAFFIC["source_sha256_16"] != h:
        # counters taken on another kernel source: reported as unknown
        assert per is None
        return
    # more than the algorithmic one read and one write of the 580 x 582 system
    assert per is not None and per > 2 * 8 * 580 * 582
