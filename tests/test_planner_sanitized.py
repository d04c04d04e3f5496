"""Host planner under AddressSanitizer and UndefinedBehaviorSanitizer.

The block-pair planner (csrc/plan.cpp) is plain C++ that turns the
block-sparse contractions of the absorption chain (Sec. 3) into offset
tables for the device kernels. ``planner_check.cpp`` builds random
block-sparse operands, plans GEMM and layer steps over them and replays every
offset a kernel would form; here it is compiled with g++ and both sanitizers
and must exit cleanly.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PLAN = os.path.join(HERE, "..", "paper_2511_01039_amd", "csrc", "plan.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_planner_offsets_under_sanitizers(tmp_path):
    exe = str(tmp_path / "planner_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-o", exe, os.path.join(HERE, "planner_check.cpp"), PLAN]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "80"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "0 failed checks" in r.stdout
