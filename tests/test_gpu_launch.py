"""Launch shapes of the sweep (btrt_set_launch / btrt_get_launch / btrt_tune).

Every shape must give the bits of one step per launch: the strip walkers over steps per launch,
strip rows and strips per group, and the two-step LDS tile, on a grid with every kind of
boundary and on a periodic one, with step counts that end in a shorter launch. The tuner runs
real steps on the live state, so after tuning the state must equal plain stepping by the
same number of steps.
"""
import sys

import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W
from tests.test_gpu_parity import custom

pytestmark = pytest.mark.gpu

# The tuner's candidate shapes: (steps_per_launch, strip_rows, strips_per_group, tile).
SHAPES = [(1, 0, 0, 0), (1, 1, 0, 0), (1, 8, 0, 0), (1, 16, 0, 0), (2, 0, 0, 1), (6, 0, 0, 0), (7, 0, 0, 0),
          (7, 61, 1, 0), (6, 342, 1, 0)] + [(k, r, g, 0) for k in (2, 3, 4, 5, 6, 7) for r in (8, 16, 32, 64, 128)
                                            for g in (1, 4)]

GRIDS = [
    custom("walls_mixed", 150, 83, 0, bc_type=(1, 1, 0, 0), bc_value=(0.3, 0.8, 0, 0), flux_b=(0.04, -0.03),
           beta=0.5, source=("sin", 0.003, 1, 2)),
    custom("periodic_aniso", 131, 70, 0, flux_b=(0.02, 0.03), beta=0.3),
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", [btrt.F64, btrt.F32, btrt.F16DEV], ids=["f64", "f32", "f16dev"])
@pytest.mark.parametrize("w", GRIDS, ids=lambda w: w.name)
def test_every_launch_shape_is_bitwise_identical(w, precision):
    steps = 2 * 4 * 3 + 1
    say(f"[gpu] launch shapes {w.name} {w.nx}x{w.ny} prec={precision} steps={steps}")
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0()) as ref:
        ref.set_fusion(1).step(steps)
        want_f, want_phi = ref.populations(), ref.field()
    for shape in SHAPES:
        with btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0()) as s:
            s.set_launch(*shape).step(steps)
            assert np.array_equal(s.populations(), want_f), shape
            assert np.array_equal(s.field(), want_phi), shape


@pytest.mark.parametrize("w", [GRIDS[0], W.c3().scaled(512, 512, 0)], ids=["walls_mixed", "c3_512"])
def test_tune_advances_the_state_like_plain_steps(w):
    say(f"[gpu] tune {w.name} {w.nx}x{w.ny}")
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        shape, used = s.tune(400)
        assert 0 < used <= 400
        assert s.info().step == used
        assert s.launch() == shape
        k, rows, group, tile = shape
        assert 1 <= k <= 7 and group in (0, 1, 4) and tile in (0, 1)
        s.step(13)
        got = s.populations()
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as r:
        r.set_fusion(1).step(used + 13)
        assert np.array_equal(r.populations(), got)


def test_tune_with_too_few_steps_keeps_the_shape():
    w = W.c1(1.0)
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        before = s.launch()
        shape, used = s.tune(1)  # no candidate (one step per launch: one untimed, one timed) fits
        assert used == 0 and shape == before and s.info().step == 0


def test_automatic_shape_by_grid_size():
    with btrt.Solver(btrt.problem_from_workload(W.c1(1.0)), W.c1(1.0).phi0()) as s:
        assert s.launch() == (1, 4, 0, 0)  # 64 x 64: one step per launch, 64 x 4 tiles
    w = W.c2()
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        k, rows, group, tile = s.launch()
        assert k == 4 and rows in (8, 16, 32) and group in (1, 4) and tile == 0
    # From 2^22 nodes: seven steps per launch, one strip per group, on periodic grids with plain
    # storage; four with 16-bit storage. FP64 seven-step walkers (one wavefront
    # per SIMD) take strips tall enough for one round over the resident slots: at 2048^2, 40
    # strips across, 82 rows (1000 strips) with 1024 slots.
    big = W.c3().scaled(2048, 2048, 0)
    for prec in (btrt.F64, btrt.F32):
        with btrt.Solver(btrt.problem_from_workload(big, precision=prec), big.phi0()) as s:
            k, rows, group, tile = s.launch()
            assert k == 7 and group == 1 and tile == 0, (prec, s.launch())
            if prec == btrt.F64:
                import torch
                cus = torch.cuda.get_device_properties(0).multi_processor_count
                assert rows >= 64 and 40 * ((2048 + rows - 1) // rows) <= cus * 4, s.launch()
            else:
                assert rows in (16, 32, 64), s.launch()
    with btrt.Solver(btrt.problem_from_workload(big, precision=btrt.F16DEV), big.phi0()) as s:
        assert s.launch()[0] == 4
    # With Dirichlet walls: six steps per launch in FP64 from 2^22 nodes (the seven-step walker
    # carries the bounce-back registers), in FP32 four below 2^24 nodes and seven from there;
    # below 2^22 nodes four.
    walled = W.c2().scaled(2048, 2048, 0)
    with btrt.Solver(btrt.problem_from_workload(walled), walled.phi0()) as s:
        assert s.launch()[0] == 6
    with btrt.Solver(btrt.problem_from_workload(walled, precision=btrt.F32), walled.phi0()) as s:
        assert s.launch()[0] == 4
    big_walled = W.c2().scaled(4096, 4096, 0)
    with btrt.Solver(btrt.problem_from_workload(big_walled, precision=btrt.F32), big_walled.phi0()) as s:
        assert s.launch()[0] == 7
    small = W.c2()
    with btrt.Solver(btrt.problem_from_workload(small), small.phi0()) as s:
        assert s.launch()[0] == 4


def test_invalid_launch_shapes_are_rejected():
    w = W.c1(1.0)
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        for bad in [(8, 0, 0, 0), (-1, 0, 0, 0), (2, -1, 0, 0), (2, 16, 3, 0), (3, 0, 0, 1), (1, 0, 0, 1),
                    (1, 3, 0, 0), (1, 32, 0, 0)]:
            with pytest.raises(btrt.BtrtError) as e:
                s.set_launch(*bad)
            assert e.value.code == btrt.E_INVAL, bad


@pytest.mark.parametrize("walls", [False, True], ids=["periodic", "walled"])
def test_single_round_strips_are_bitwise_identical(walls):
    # FP64 walkers from six steps per launch hold one wavefront per SIMD; their automatic strips
    # are tall enough for one round over the resident slots only on large grids (2048^2: 40 strips
    # across, 82 rows at K = 7), so the small grids above never take them. 15 steps: two 7-step
    # launches and a 1-step one, or two 6-step launches and a 3-step one.
    w = W.c3().scaled(2048, 2048, 0)
    if walls:
        w = W.Workload("walled_2048", 2048, 2048, 0, flux_b=w.flux_b, A0=w.A0, beta=w.beta, bc_type=(1, 1, 1, 1),
                       bc_value=(0.2, -0.1, 0.5, 0.3), seed=11, phi0_kind="uniform")
    steps = 15
    say(f"[gpu] single-round strips {w.name} {w.nx}x{w.ny}, {steps} steps")
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0(), torch_memory=True) as ref:
        ref.set_launch(1, 4, 1, 0).step(steps)
        want = ref.populations()
    for k in (6, 7):
        with btrt.Solver(btrt.problem_from_workload(w), w.phi0(), torch_memory=True) as s:
            s.set_launch(k, 0, 0, 0)
            _, rows, group, _ = s.launch()
            assert rows >= 64 and group == 1, s.launch()
            s.step(steps)
            assert np.array_equal(s.populations(), want), (k, rows)
