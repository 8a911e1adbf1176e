"""bench.py's contract on the CPU: a one-GPU build that refuses N > 1, the
algorithmic byte counts its roofline uses, and committed counter records
that still describe the committed kernels (a stale record would make the
benchmark report null traffic and VALU figures)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_node():
    # displacement read (8 d) + each value read and written (2 s nf); the fused
    # launch also writes the next step's displacement (8 d)
    assert bench.recon_bytes_per_node(2, 3, 4) + bench.traj_bytes_per_node(2) == 56
    assert bench.recon_bytes_per_node(3, 3, 4) + bench.traj_bytes_per_node(3) == 72
    assert bench.recon_bytes_per_node(3, 1, 8) + bench.traj_bytes_per_node(3) == 64
    assert bench.recon_bytes_per_node(2, 3, 8) == 64


@pytest.mark.parametrize("key,alg", [
    # 64 B x 512^3 (FP64 value, 3-D displacement read and next one written)
    (("deform3d", 512, "f64"), 64 * 512 ** 3),
    # 56 B x 1024^2 (three FP32 values, 2-D displacements)
    (("swirl", 1024, "f32"), 56 * 1024 ** 2),
])
def test_traffic_records_match_the_kernels(key, alg):
    t = bench.recorded_traffic(key)
    assert t is not None, "profiles/ traffic record of %s is stale: re-take it" % (key,)
    # within a few percent of the algorithmic bytes (the limiter's order
    # words add 2 B per node)
    assert 0.9 < t / alg < 1.5


def test_headline_is_the_largest_single_gpu_configuration():
    assert bench.HEADLINE == ("deform3d", 512, "f64")
    assert bench.HEADLINE in bench.TRAFFIC


@pytest.mark.parametrize("key", [
    "swirl_f32/recon2d_tiled_kernel<float, 3, 2>",
    "fourier3d_f32/recon3d_kernel<float, 3, 4>",
    "deform3d_f64/recon3d_kernel<double, 1, 3>",
    "deform3d_f32/recon3d_kernel<float, 1, 3>",
    "kelvin_f64/recon2d_tiled_kernel<double, 3, 6>",
    "kelvin_f64/sw_stage_kernel<double, 2>",
])
def test_valu_record_matches_the_kernels(key):
    r = bench.valu_roof(key, 1.0)
    assert r is not None, "profiles/ VALU record is stale or lacks %s" % key
    assert r["bound"] == "alu" and r["valu_per_wave"] > 100 and r["waves"] > 0
    # the peak is 1024 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction
    assert abs(r["peak"] - 1024 * 2.4e9 / 4) < 1.0
