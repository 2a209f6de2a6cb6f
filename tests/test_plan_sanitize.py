"""The host plan builders (window plan, launch tables, pose-graph plan) built
with AddressSanitizer and UndefinedBehaviorSanitizer and run on seeded random
structures, including inputs that the validation must reject; every packed
field of the launch tables is decoded and checked (tests/native/plan_check.cpp).
Host code only: no GPU, no HIP."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_04359_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_plan_builders_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "plan_check.cpp"),
           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "pgo_plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "60"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "0 failures" in r.stdout and "windows" in r.stdout, r.stdout
