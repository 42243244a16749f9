"""The host planner (tree, boxes, Gauss bookkeeping, refined interfaces) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on
uniform, rectangular, multi-problem and refined trees; its invariants are
checked by the driver (tests/planner_sanitize.cpp)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1612_02736_amd", "csrc")


def test_planner_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "planner_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(HERE, "planner_sanitize.cpp"), os.path.join(CSRC, "plan.cpp"),
           os.path.join(CSRC, "spectral.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    # the environment is passed on unchanged apart from the sanitizer options
    # (a library preloaded by the environment need not come after ASan's)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr
