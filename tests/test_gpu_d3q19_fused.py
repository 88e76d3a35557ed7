"""Two time steps per D3Q19 launch (btrt3_set_launch): the same bits as one step per launch.

Every tile shape (64 x 8, 32 x 16, 32 x 8 and 16 x 16 threads) and a range of z chunks (1, 2, 3, 7 planes, larger
than the box, automatic) on periodic boxes, boxes with Dirichlet faces on some or all axes,
ragged boxes narrower than a tile, one-node-thick slabs, a phi-dependent tensor and a source
field, in FP64 and FP32; odd step counts (the last launch takes one step) and split calls. The
automatic shape of a grid from 2^21 nodes up is the two-step launch. One FP64 case is also held
against the oracle directly (1e-12 normwise).
"""
import sys

import numpy as np
import pytest

from paper_1902_09813_amd import btrt, btrt3
from paper_1902_09813_amd import workloads as W
from tests._cases import normwise, run_oracle3

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _box(nx, ny, nz, bc, steps=21, beta=0.3, source=False, seed=0):
    rng = np.random.default_rng(seed + nx * 1000 + ny * 10 + nz)
    src = 1e-3 * rng.standard_normal((nz, ny, nx)) if source else None
    return W.Workload3(f"d3_{nx}x{ny}x{nz}_{''.join(map(str, bc))}{'_src' if source else ''}", nx, ny, nz, steps,
                       flux_a=(0.02, -0.03, 0.01), flux_b=(0.01, 0.0, 0.02),
                       A0=(0.04, 0.005, 0.0, 0.03, -0.004, 0.05), beta=beta, source=src, bc_type=bc,
                       bc_value=(0.3, 0.1, 0.7, 0.2, 0.5, 0.4), k2=1.1, k0=0.9,
                       phi0_array=rng.random((nz, ny, nx)))


CASES = [_box(37, 23, 9, (0,) * 6), _box(37, 23, 9, (1,) * 6), _box(33, 30, 12, (1, 1, 0, 0, 1, 1), source=True),
         _box(5, 40, 17, (0, 0, 1, 1, 0, 0), beta=0.0), _box(20, 7, 30, (1, 1, 1, 1, 0, 0)),
         _box(1, 1, 1, (0,) * 6), _box(1, 1, 1, (1,) * 6), _box(9, 7, 1, (1, 1, 1, 1, 0, 0)),
         _box(15, 1, 11, (0, 0, 1, 1, 1, 1)), W.d3_walls(), W.d3_nonlinear(24, 19, 13, steps=21)]
SHAPES = [(2, 1, 1), (2, 2, 2), (2, 3, 3), (2, 7, 4), (2, 64, 1), (2, 0, 0), (2, 0, 4), (2, 5, 2), (2, 0, 3)]


def run(w, shape, steps, precision=btrt.F64, split=None):
    with btrt3.Solver3(btrt3.problem_from_workload3(w, precision=precision), w.phi0()) as s:
        s.set_launch(*shape)
        if split:
            s.step(split).step(steps - split)
        else:
            s.step(steps)
        assert s.info().step == steps
        return s.populations(), s.field()


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_two_steps_per_launch_bitwise_fp64(w):
    f1, p1 = run(w, (1, 0, 0), w.steps)
    for shape in SHAPES:
        say(f"[gpu] d3q19 two-step {w.name} shape={shape} steps={w.steps}")
        f2, p2 = run(w, shape, w.steps)
        assert np.array_equal(f1, f2) and np.array_equal(p1, p2), shape


@pytest.mark.parametrize("w", [CASES[0], CASES[2], CASES[4]], ids=lambda w: w.name)
def test_two_steps_per_launch_bitwise_fp32(w):
    f1, _ = run(w, (1, 0, 0), w.steps, btrt.F32)
    for shape in [(2, 3, 0), (2, 0, 2), (2, 4, 3)]:
        say(f"[gpu] d3q19 two-step f32 {w.name} shape={shape}")
        f2, _ = run(w, shape, w.steps, btrt.F32)
        assert np.array_equal(f1, f2), shape


def test_split_calls_and_odd_counts():
    w = CASES[1]
    f1, _ = run(w, (1, 0, 0), 20)
    for split in (1, 2, 7):
        f2, _ = run(w, (2, 5, 0), 20, split=split)
        assert np.array_equal(f1, f2), split


def test_two_step_launch_against_the_oracle():
    w = _box(30, 17, 16, (1, 1, 0, 0, 1, 1), steps=30, source=True)
    f, phi = run(w, (2, 4, 1), w.steps)
    o = run_oracle3(w)
    e_phi, e_f = normwise(phi, o.phi()), normwise(f, o.f)
    say(f"    two-step vs oracle: normwise phi {e_phi:.3e}  f {e_f:.3e}")
    assert e_phi <= 1e-12 and e_f <= 1e-12


def test_automatic_shape_is_two_steps_from_2_21_nodes():
    w = W.d3_nonlinear(128, 128, 128, steps=5)
    with btrt3.Solver3(btrt3.problem_from_workload3(w), w.phi0()) as s:
        k, zc, tile = s.launch()
        assert k == 2 and 16 <= zc <= 128 and tile == 1
        s.step(w.steps)
        f2 = s.populations()
    with btrt3.Solver3(btrt3.problem_from_workload3(w), w.phi0()) as s:
        s.set_launch(1)
        assert s.launch()[0] == 1
        s.step(w.steps)
        assert np.array_equal(s.populations(), f2)
    small = CASES[0]
    with btrt3.Solver3(btrt3.problem_from_workload3(small), small.phi0()) as s:
        assert s.launch()[0] == 1


def test_invalid_launch_shapes_are_rejected():
    w = CASES[5]
    with btrt3.Solver3(btrt3.problem_from_workload3(w), w.phi0()) as s:
        for bad in [(3, 0, 0), (-1, 0, 0), (2, -1, 0), (2, 0, 5), (2, 0, -1)]:
            with pytest.raises(btrt.BtrtError) as e:
                s.set_launch(*bad)
            assert e.value.code == btrt.E_INVAL, bad
