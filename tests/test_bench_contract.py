"""The benchmark's command-line contract and its use of the committed profile
summaries (host only)."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_bench_help():
    r = run_bench("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--precision", "--lattice", "--one-stream"):
        assert flag in r.stdout


def test_bench_refuses_several_gpus():
    """The measured path runs on one GPU: --gpus above 1 exits with a message
    (before anything touches a device)."""
    r = run_bench("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def fields(path):
    out = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


@pytest.mark.parametrize("kernel", ["k_rt_f64", "k_gemm_f64"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_profile_traffic_only_for_current_source(kernel, precision):
    """An HBM-traffic summary names the kernel source it was taken from and
    that file's hash; the benchmark reports its traffic figure only while the
    hash is that of the current source, and null once the kernel changed."""
    sys.path.insert(0, ROOT)
    import bench
    path = os.path.join(ROOT, "profiles", f"{kernel}_config4_{precision}_hbm_traffic.txt")
    if not os.path.exists(path):
        assert bench.profiled_traffic(kernel, precision) is None
        return
    f = fields(path)
    src = os.path.join(ROOT, f["kernel_source"])
    fresh = hashlib.sha256(open(src, "rb").read()).hexdigest() == f["kernel_source_sha256"]
    got = bench.profiled_traffic(kernel, precision)
    if fresh:
        assert got == float(f["traffic_bytes_per_launch"]) and got > 0
    else:
        assert got is None


def test_profiles_name_their_commands():
    """Every summary under profiles/ gives the command that produced it."""
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "rocprofv3" in text and "bench.py" in text, name
