"""The oracle under gcc's address and undefined-behaviour sanitizers (host
only): oracle/asan_check.c links psd_oracle.c into an instrumented program
that runs the projection, its derivative and pack/unpack (OpenMP on) on small orders in
both Jacobi orderings and checks their identities; any out-of-bounds access,
use after free, leak or undefined operation aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_asan")
    flags = ["-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    cmd = [gcc, *flags, "-std=gnu11", "-o", exe, os.path.join(ROOT, "oracle", "psd_oracle.c"),
           os.path.join(ROOT, "oracle", "asan_check.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("no sanitizer runtime: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout + run.stderr)[-2000:]
    assert run.stdout.strip().endswith("ok")
