"""Host-side logic of bench.py (no GPU): the one-GPU contract, the count of sweep launches the
timed region makes, and the lookup of the committed HBM counter record."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_sweep_launch_count():
    # Chunks of the residual check interval (1000 steps), each ending in a shorter launch when the
    # steps per launch do not divide it.
    assert bench.sweep_launches(5000, 1) == 5000
    assert bench.sweep_launches(5000, 4) == 5 * 250
    assert bench.sweep_launches(5000, 7) == 5 * (142 + 1)
    assert bench.sweep_launches(2500, 6) == 2 * (166 + 1) + (83 + 1)
    assert bench.sweep_launches(0, 7) == 0


def test_traffic_record_lookup():
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    nodes = 4096 * 4096
    if rec["kernel_sha256_16"] != bench.kernel_hash():
        # Counters taken on other kernel sources: the benchmark must report no traffic.
        assert bench.traffic_for("f64", nodes, dict(steps_per_launch=7, strip_rows=64, strips_per_group=1,
                                                    tile=0)) is None
        pytest.skip("the HBM counter record predates the current kernel sources")
    shape = dict(steps_per_launch=7, strip_rows=64, strips_per_group=1, tile=0)
    got = bench.traffic_for("f64", nodes, shape)
    alg = 160 * nodes
    assert got is not None and alg <= got <= 1.3 * alg
    busy = bench.valu_busy_for("f64", nodes, shape)
    assert busy is not None and 0.0 < busy <= 1.0
    assert bench.valu_busy_for("f64", nodes, dict(shape, strip_rows=8)) is None
    assert bench.traffic_for("f64", nodes + 1, shape) is None  # another grid
    assert bench.traffic_for("f64", nodes, dict(shape, strip_rows=8)) is None  # a shape not measured
    assert bench.traffic_key("f32", dict(steps_per_launch=4, strip_rows=32, strips_per_group=4, tile=0)) == \
        "f32_k4_r32_g4_t0"
