"""The runtime's host code under the address and undefined-behaviour
sanitizers, without a GPU: every translation unit of the library is compiled
with the sanitizers on its host code only (the device code is built as usual), linked with
tests/host_asan_check.cpp, and run.  The program drives the entry points
along every path that ends on the host (layouts of single blocks, cones and
SCS settings; argument validation; the cleanup of calls whose first device
call fails here), so an out-of-bounds access, use after free or undefined
operation in that code aborts it."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-I" + os.path.join(ROOT, "include")]


def test_runtime_host_code_under_address_sanitizer(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2606_20519_amd", "csrc", "*.hip")))
    srcs.append(os.path.join(ROOT, "tests", "host_asan_check.cpp"))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src).split(".")[0] + ".o"))
        r = subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
        return obj, r.returncode, r.stderr

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, srcs))
    for obj, rc, err in results:
        assert rc == 0, err[-2000:]
    exe = str(tmp_path / "host_asan_check")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                        "-fsanitize=undefined",
                        *[o for o, _, _ in results], "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    # leaks are not checked: the HIP runtime keeps its own allocations to exit
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    assert "runtime error" not in run.stderr, run.stderr[-3000:]
    assert run.stdout.strip().endswith("ok")
