"""bench.py's host-side contract, without a GPU: more than one GPU is
refused with a message; the HBM traffic of the dominant kernel is taken from
the committed counter summary only while the kernel's sources still have the
hash recorded with it (so the committed summary and the committed HEMV
kernel agree); the algorithmic flop counts follow the stated formulas."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    assert "one GPU" in json.loads(line)["error"]


def test_committed_traffic_matches_committed_kernel():
    t = bench.measured_traffic("hemv_kernel", 4096, ("tridiag.hip", "common.h"))
    assert t is not None and t > 0
    assert bench.measured_traffic("hemv_kernel", 4096, ("tridiag.hip", "gemm.hip")) is None  # other sources


def test_flop_formulas():
    n, k = 4096, 2048
    assert bench.flops_eig(n, k) == 16.0 / 3.0 * n ** 3 + 12.0 * n * n * k
    assert bench.flops_ns(n, 12, 1) == 12 * 8.0 * n ** 3 + 8.0 * n ** 3 + 8.0 * n ** 3
