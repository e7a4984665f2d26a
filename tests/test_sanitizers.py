"""The host symbolic analysis (integer work on the block graph) built with
AddressSanitizer and UndefinedBehaviorSanitizer by the host compiler and run
on several grids, both elimination orders, both coarsenings, a general
graph and a joined batch of 2D and 3D problems (with invalid ones that must
be reported); every access out of bounds, use after free, overflow or other
undefined behaviour aborts the driver (CPU only, no HIP involved)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1603_09133_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_symbolic_analysis_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "symbolic_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", CSRC,
           os.path.join(CSRC, "symbolic.cpp"), os.path.join(ROOT, "tests", "native", "symbolic_check.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
