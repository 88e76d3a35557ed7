"""Checkpoint and resume through the C ABI (btrt_checkpoint / btrt_restore).

* A run interrupted at any step and restored into a new handle of the same problem continues
  with exactly the bits of the uninterrupted run, in every storage format, across launch shapes
  (the restored handle may use another shape), and with the Eq. (64) snapshot carried over.
* The Burgers-Fisher variant: a checkpoint under a wall schedule restores the values in force;
  with the rest of the schedule set again the result equals the uninterrupted run.
* A checkpoint is refused (BTRT_E_INVAL, state untouched) by a handle of another grid, precision
  or problem constant, and a buffer that is not a checkpoint or is too short is refused.
"""
import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W

pytestmark = pytest.mark.gpu


def case(nx=131, ny=70):
    return W.Workload("ck_walls", nx, ny, 0, A0=(0.03, 0.006, 0.02), beta=0.5, flux_a=(0.03, -0.02),
                      flux_b=(0.02, 0.0), source=("sin", 2e-3, 1, 1), bc_type=(1, 1, 1, 1),
                      bc_value=(0.2, 0.6, 0.4, 0.1), seed=21)


@pytest.mark.parametrize("precision", [btrt.F64, btrt.F32, btrt.F16DEV, btrt.BF16DEV],
                         ids=["f64", "f32", "f16dev", "bf16dev"])
def test_resume_is_bitwise(precision):
    w = case()
    n1, n2 = 37, 53
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision, check_interval=10), w.phi0()) as ref:
        ref.set_launch(4, 16, 4, 0).step(n1)
        r1 = ref.residual()
        ref.step(n2)
        want_f, want_r = ref.populations(), ref.residual()
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision, check_interval=10), w.phi0()) as a:
        a.set_launch(4, 16, 4, 0).step(n1)
        assert a.residual() == r1
        data = a.checkpoint()
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision, check_interval=10), w.phi0()) as b:
        b.set_launch(6, 32, 1, 0)  # another shape: the same bits
        b.restore(data)
        assert b.info().step == n1
        b.step(n2)
        assert np.array_equal(b.populations(), want_f)
        assert b.residual() == want_r  # the snapshot came along


def test_resume_under_a_wall_schedule():
    w = W.bfe(n=20, alpha=0.05, t_end=1.0)
    n1, n2 = 41, 59
    sched = btrt.wall_schedule(w, 0, n1 + n2)
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as ref:
        ref.set_walls(sched).step(n1 + n2)
        want = ref.populations()
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as a:
        a.set_walls(sched[:n1]).step(n1)
        data = a.checkpoint()
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as b:
        b.restore(data)
        with pytest.raises(btrt.BtrtError):
            b.step(1)  # the rest of the schedule is not set yet
        b.set_walls(sched[n1:]).step(n2)
        assert np.array_equal(b.populations(), want)
    # Into a handle of the plain problem (no general model): it switches to the wall table.
    wc = W.Workload("walls_table", 40, 30, 0, A0=(0.03, 0.0, 0.02), flux_a=(0.02, 0.01), bc_type=(1, 1, 1, 1),
                    bc_value=(0.1, 0.2, 0.3, 0.4), seed=3)
    rows = np.random.default_rng(1).uniform(0.0, 1.0, (30, 4 * (40 + 30) + 4))
    with btrt.Solver(btrt.problem_from_workload(wc), wc.phi0()) as ref:
        ref.set_walls(rows).step(30)
        want = ref.populations()
    with btrt.Solver(btrt.problem_from_workload(wc), wc.phi0()) as a:
        a.set_walls(rows[:12]).step(12)
        data = a.checkpoint()
    with btrt.Solver(btrt.problem_from_workload(wc), wc.phi0()) as b:
        b.restore(data).set_walls(rows[12:]).step(18)
        assert np.array_equal(b.populations(), want)


def test_mismatches_are_refused():
    w = case()
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as a:
        a.step(5)
        data = a.checkpoint()
    others = [case(nx=130), case(ny=71)]
    other = case()
    other.bc_value = (0.2, 0.6, 0.4, 0.11)
    others.append(other)
    other = case()
    other.beta = 0.6
    others.append(other)
    for o in others:
        with btrt.Solver(btrt.problem_from_workload(o), o.phi0()) as b:
            before = b.populations()
            with pytest.raises(btrt.BtrtError) as e:
                b.restore(data)
            assert e.value.code == btrt.E_INVAL
            assert b.info().step == 0 and np.array_equal(b.populations(), before)
    with btrt.Solver(btrt.problem_from_workload(w, precision=btrt.F32), w.phi0()) as b:
        with pytest.raises(btrt.BtrtError):
            b.restore(data)
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as b:
        for bad in (data[:100], data[:-8], b"x" * len(data)):
            with pytest.raises(btrt.BtrtError) as e:
                b.restore(bad)
            assert e.value.code == btrt.E_INVAL
