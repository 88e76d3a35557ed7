"""Batched solves (btrt_batch_*): many uneven instances in one launch per step.

Every instance of a batch must give the bits it gives when solved alone (btrt_create /
btrt_step), for every launch configuration, with graph replay, after the autotuner, and it
must match the FP64 oracle to 1e-12 normwise.
"""
import sys

import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W
from tests._cases import normwise, run_oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_mix(count=24, precision=btrt.F64, seed=4):
    """Seeded uneven instances like the 256-instance workload, with sides 8..150 (oracle speed)."""
    ws = W.c4(count=count, seed=seed, steps=0, side_range=(8, 150))
    # Make some instances rectangular and one degenerate (1 x n) to exercise ragged tiles.
    ws[1].nx = max(1, ws[1].nx // 3)
    ws[2].ny = 1
    return [(btrt.problem_from_workload(w, precision=precision), w.phi0()) for w in ws], ws


def alone(problem, phi0, steps, fusion=2):
    with btrt.Solver(problem, phi0) as s:
        s.set_fusion(fusion).step(steps)
        return s.field()


@pytest.mark.parametrize("precision", [btrt.F64, btrt.F32], ids=["f64", "f32"])
def test_batch_equals_each_instance_alone(precision):
    probs, ws = small_mix(precision=precision)
    steps = 37
    say(f"[gpu] batch of {len(probs)} instances, {steps} steps, precision {precision}")
    with btrt.Batch(probs) as b:
        b.step(steps)
        got = [b.field(i) for i in range(b.n)]
    for i, (p, ph) in enumerate(probs):
        ref = alone(btrt.problem_from_workload(ws[i], precision=precision), ph, steps)
        assert np.array_equal(got[i], ref), ws[i].name


@pytest.mark.parametrize("cfg", [(1, 0, 0, 0), (2, 0, 0, 0), (2, 2, 0, 0), (1, 8, 0, 0), (2, 8, 0, 0), (2, 0, 4, 0),
                                 (1, 2, 16, 0), (2, 4, 16, 0), (4, 0, 0, 16), (4, 0, 0, 5), (4, 4, 0, 32),
                                 (4, 2, 16, 8), (4, 0, 4, 16), (6, 0, 0, 16), (6, 0, 4, 32), (7, 0, 0, 16),
                                 (7, 0, 2, 32), (7, 4, 0, 8)], ids=lambda c: "s%d_b%d_g%d_r%d" % c)
def test_batch_configurations_bitwise_identical(cfg):
    # 4-, 6- and 7-step strip walkers included: step counts that are not multiples of k end with
    # 2- and 1-step launches; graph replays of k-step launches; strips shorter than the instances.
    probs, _ = small_mix(count=16, seed=41)
    steps = 70
    with btrt.Batch(probs) as ref_b, btrt.Batch(probs) as b:
        ref_b.set_config(1, 0, 0).step(steps)
        b.set_config(*cfg)
        # Several calls, with eager work (a residual) between graph replays.
        for k in (33, 0, 21, 16):
            b.step(k)
            b.residual()
        ref_b.residual()
        assert b.steps() == ref_b.steps() == steps
        for i in range(b.n):
            assert np.array_equal(b.field(i), ref_b.field(i))


def test_batch_residuals_match_single_solves():
    probs, ws = small_mix(count=10, seed=7)
    with btrt.Batch(probs) as b:
        b.step(120)
        r1 = b.residual()
        b.step(80)
        r2 = b.residual()
    for i, (p, ph) in enumerate(probs):
        with btrt.Solver(btrt.problem_from_workload(ws[i]), ph) as s:
            s.step(120)
            assert s.residual() == r1[i]
            s.step(80)
            assert s.residual() == r2[i]


def test_batch_autotuner_keeps_the_solution():
    probs, _ = small_mix(count=12, seed=9)
    with btrt.Batch(probs) as b, btrt.Batch(probs) as ref_b:
        best, used = b.tune(2000)
        say(f"    tuned config {best} after {used} steps")
        assert used <= 2000 and b.config() == best
        b.step(101)
        ref_b.step(used + 101)
        for i in range(b.n):
            assert np.array_equal(b.field(i), ref_b.field(i))


def test_batch_fp64_matches_oracle():
    probs, ws = small_mix(count=8, seed=13)
    steps = 150
    with btrt.Batch(probs) as b:
        b.step(steps)
        for i, w in enumerate(ws):
            w.steps = steps
            e = normwise(b.field(i), run_oracle(w).phi())
            assert e <= 1e-12, (w.name, e)


def test_full_batched_workload_sampled_against_alone():
    # The 256-instance FP32 workload, 2000 steps, tuned; a sample of instances solved alone.
    ws = W.c4()
    probs = [(btrt.problem_from_workload(w, precision=btrt.F32), w.phi0()) for w in ws]
    say(f"[gpu] full batched workload: {len(ws)} instances, {sum(w.nx * w.ny for w in ws)} nodes")
    with btrt.Batch(probs) as b:
        best, used = b.tune(1200)
        say(f"    tuned config {best} after {used} steps")
        assert used > 0
        b.step(2000 - used)
        assert b.steps() == 2000
        res = b.residual()
        assert np.all(np.isfinite(res))
        for i in (0, 1, 17, 100, 255):
            ref = alone(btrt.problem_from_workload(ws[i], precision=btrt.F32), probs[i][1], 2000)
            assert np.array_equal(b.field(i), ref), ws[i].name


def test_batch_rejects_unsupported_steps_per_launch():
    probs, _ = small_mix(count=4, seed=3)
    with btrt.Batch(probs) as b:
        for bad in (3, 5, 8, 0, -1):
            with pytest.raises(btrt.BtrtError) as e:
                b.set_config(bad, 0, 0)
            assert e.value.code == btrt.E_INVAL, bad
