"""The benchmark's host-side contract, on the CPU: one GPU only, and the
algorithmic bytes per node that the roofline figure is built on."""
import functools
import os
import subprocess
import sys

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@functools.lru_cache(maxsize=None)
def workload(name):
    return bench.make_workload(name)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


@pytest.mark.parametrize("name,bpn", [
    # every population read and written once, plus the history (u, phi, c1, c2)
    ("static_drop_64x64", 2 * 36 * 8 + 2 * 5 * 8),                  # FP64, D2Q9 x 4
    ("rising_bubble_256x1024", 2 * 36 * 4 + 2 * 5 * 4),             # FP32, D2Q9 x 4
    ("rising_droplet_256c_f32", 2 * 40 * 4 + 2 * 6 * 4),            # FP32, D3Q19 + 3 x D3Q7
    ("rising_droplet_256c_f32_s16f", 2 * 40 * 2 + 2 * 6 * 4),       # 16-bit populations
    ("rising_bubble_one_256x1024", 2 * 27 * 4 + 2 * 4 * 4),         # one-scalar: f, g, h3
])
def test_algorithmic_bytes_per_node(name, bpn):
    assert bench.alg_bytes_per_node(workload(name)["params"]) == bpn


def test_workload_sizes():
    assert W.n_nodes(workload("rising_bubble_256x1024")["params"]) == 256 * 1024
    assert W.n_nodes(workload("rising_droplet_256c_f32")["params"]) == 256 ** 3
