"""Host-side checks of bench.py: the one-GPU refusal, the digest that ties
the stored HBM traffic to the kernel sources, and the price list that turns
the oracle's event counts into flops per point.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [0, 2, 8])
def test_bench_refuses_other_gpu_counts(n):
    """The bench measures one GPU; any other count exits with status 2 and a
    message on stderr, and prints no JSON line."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert r.stdout.strip() == ""
    assert "one GPU" in r.stderr and ("--gpus %d" % n) in r.stderr


def test_kernel_digest_covers_existing_sources():
    """The digest reads every listed kernel source, and changes with them:
    the stored traffic is reported only for the sources it was measured on."""
    for f in bench.KERNEL_SOURCES:
        assert os.path.isfile(os.path.join(ROOT, "paper_2309_13824_amd", "csrc", f)), f
    d = bench.kernel_digest()
    assert len(d) == 40 and int(d, 16) >= 0
    assert d == bench.kernel_digest()


def test_flops_price_list():
    """No events: only the fixed per-point part (extraction and statistics).
    One of each event adds its own price once; the prices are linear."""
    zero = {k: 0 for k in bench.FLOPS_PER_EVENT}
    assert bench.flops_per_point(zero) == bench.FLOPS_PER_POINT_FIXED
    for k, price in bench.FLOPS_PER_EVENT.items():
        one = dict(zero, **{k: 1.0})
        assert bench.flops_per_point(one) - bench.FLOPS_PER_POINT_FIXED == price
    mix = {"candidates": 22.0, "clip_tests": 45.0, "cuts": 6.0, "vertices": 6.0, "quad_points": 10.0}
    expect = bench.FLOPS_PER_POINT_FIXED + 5 * 22 + 4 * 45 + 20 * 6 + 3 * 6 + 27 * 10
    assert bench.flops_per_point(mix) == expect


def test_algorithmic_bytes_per_point():
    """The FP64 figure differs from the FP32 one only by the wider positions
    read in the cell scan (4 bytes per point)."""
    assert bench.BYTES_PER_POINT["fp64"] - bench.BYTES_PER_POINT["fp32"] == 4
    assert bench.BYTES_PER_POINT["fp32"] == 218


def test_cpu_info_names_the_host():
    """The CPU baseline records the model name and, where /proc/cpuinfo has
    them, the family, model and stepping numbers."""
    info = bench.cpu_info()
    assert info["model"]
    assert 1 <= info["threads_all"] <= 16
    assert info["threads_all"] <= info["cpus_available"]
    if os.path.exists("/proc/cpuinfo"):
        assert "cpu family" in info["cpu_id"] or info["cpu_id"] == ""
