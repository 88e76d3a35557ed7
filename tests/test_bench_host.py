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
        assert bench.traffic_for("f64", nodes, dict(steps_per_launch=7, strip_rows=342, strips_per_group=1,
                                                    tile=0)) is None
        pytest.skip("the HBM counter record predates the current kernel sources")
    # The tuned shape of the FP64 workload: seven steps, strips tall enough for one round.
    shape = dict(steps_per_launch=7, strip_rows=342, strips_per_group=1, tile=0)
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


def _run(k, us, nodes=4096 * 4096, tile=0):
    return {"launch": dict(steps_per_launch=k, strip_rows=64, strips_per_group=1, tile=tile), "launch_ms_avg": us * 1e-3,
            "nodes": nodes, "bytes_per_node_launch": 160.0}


def test_roofline_bound_follows_the_launch_shape():
    # One step per launch: HBM-bound, algorithmic bytes per launch over 8 TB/s.
    r1 = bench.roofline_of(_run(1, 495.0), "f64")
    assert r1["bound"] == "hbm" and r1["unit"] == "GB/s"
    assert r1["achieved"] == pytest.approx(160 * 4096 * 4096 / 495e-6 / 1e9, rel=1e-3)
    assert r1["frac"] == pytest.approx(r1["achieved"] / 8000.0, rel=1e-3)
    # Seven steps per launch: the FP64 arithmetic of 7 node updates per node bounds the launch;
    # the per-launch HBM view stays beside it and every fraction is of a bound that holds.
    r7 = bench.roofline_of(_run(7, 700.0), "f64")
    assert r7["bound"] == "alu" and r7["unit"] == "TFLOP/s" and r7["peak"] == 78.6
    flops = bench.FLOPS_PER_UPDATE * 7 * 4096 * 4096 / 700e-6 / 1e12
    assert r7["achieved"] == pytest.approx(flops, rel=1e-3)
    assert 0 < r7["frac"] < 1 and 0 < r7["fp64_issue"]["frac"] < 1 and 0 < r7["hbm_per_launch"]["frac"] < 1
    assert r7["per_update_vs_one_step_hbm_roofline"] == pytest.approx(160 * 7 * 4096 * 4096 / 700e-6 / 8e12, rel=1e-3)
    # FP32 storage: the VALU issue of the lane-instructions the counter record counted for the
    # shape when it covers it (the measured seven-step shape, on the current sources), else the
    # per-launch HBM view.
    r32 = bench.roofline_of(_run(7, 400.0), "f32")
    lanes = bench.valu_lanes_for("f32", 4096 * 4096, r32["launch"])
    if lanes is None:
        assert r32["bound"] == "hbm"
    else:
        assert r32["bound"] == "alu" and r32["unit"] == "T lane-instructions/s" and r32["peak"] == 39.3
        assert r32["achieved"] == pytest.approx(lanes * 7 * 4096 * 4096 / 400e-6 / 1e12, rel=1e-3)
    unmeasured = _run(7, 400.0)
    unmeasured["launch"]["strip_rows"] = 8
    assert bench.roofline_of(unmeasured, "f32")["bound"] == "hbm"
