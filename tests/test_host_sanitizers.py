"""The host-side setup (splines, 1D matrices, tau, eigendecompositions, FD
data, gather tables, geometry maps) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the CPU and run over uniform, graded,
repeated-knot and mapped knot vectors of degrees 1..3 (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_setup_under_asan_ubsan(tmp_path):
    exe = tmp_path / "host_setup_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", os.path.join(ROOT, "tests", "sanitize", "host_setup_check.cpp"),
           os.path.join(ROOT, "paper_2311_17500_amd", "csrc", "host_setup.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("(0 failures)")
