"""btrt_solve_static, the entry point that allocates nothing, against btrt_create + btrt_solve +
btrt_field on the same arguments: the same bits, on two calls in a row (the second on a smaller
grid, so the fixed array holds the larger call's leftovers), in FP64 and FP32, with walls, a
source and a nonlinear diffusion tensor; the FP64 result also against the oracle (1e-12
normwise). Grids too large for the array, and a workspace argument, are refused."""
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


def walled(nx, ny, steps):
    return W.Workload(f"static_walls_{nx}x{ny}", nx, ny, steps, A0=(0.03, 0.006, 0.02), beta=0.5, flux_a=(0.03, -0.02),
                      flux_b=(0.02, 0.0), source=("sin", 2e-3, 1, 1), bc_type=(1, 1, 1, 1),
                      bc_value=(0.2, 0.6, 0.4, 0.1), k0=0.9, k2=(1.1, 0.95, 0.95, 1.2), seed=21)


def periodic(nx, ny, steps):
    return W.Workload(f"static_periodic_{nx}x{ny}", nx, ny, steps, flux_b=(0.05, 0.05), A0=(0.01, 0.0, 0.005),
                      beta=1.0, seed=3, phi0_kind="gaussians", extra={"count": 16})


def by_handle(w, precision, tol, max_steps, interval):
    p = btrt.problem_from_workload(w, precision=precision, check_interval=interval)
    with btrt.Solver(p, w.phi0()) as s:
        steps, res = s.solve(tol, max_steps)
        return s.field(), steps, res


@pytest.mark.parametrize("precision", [btrt.F64, btrt.F32], ids=["f64", "f32"])
def test_two_calls_match_the_handle(precision):
    # (workload, tol, max_steps, check interval): the first stops on the tolerance, the second
    # runs out of steps.
    calls = [(walled(251, 197, 0), 5e-3, 4000, 250), (periodic(96, 70, 0), 0.0, 1300, 500)]
    for w, tol, max_steps, interval in calls:
        say(f"[gpu] static solve {w.name} precision {precision} tol {tol} max {max_steps}")
        p = btrt.problem_from_workload(w, precision=precision, check_interval=interval)
        phi, steps, res = btrt.solve_static(p, w.phi0(), tol, max_steps)
        want, want_steps, want_res = by_handle(w, precision, tol, max_steps, interval)
        say(f"    steps {steps} residual {res:.3e} (handle {want_steps}, {want_res:.3e})")
        assert steps == want_steps and res == want_res
        assert (steps < max_steps) == (tol > 0)  # the first call stops on the tolerance
        assert np.array_equal(phi, want)
        if precision == btrt.F64:
            w.steps = steps
            e = normwise(phi, run_oracle(w).phi())
            say(f"    normwise against the oracle {e:.3e}")
            assert e <= 1e-12


def test_refusals():
    big = periodic(1024, 1024, 0)
    p = btrt.problem_from_workload(big)
    assert p.workspace_size() > btrt.STATIC_BYTES
    with pytest.raises(btrt.BtrtError) as e:
        btrt.solve_static(p, big.phi0(), 0.0, 10)
    assert e.value.code == btrt.E_INVAL and "btrt_solve_static holds" in str(e.value)
    small = periodic(32, 32, 0)
    q = btrt.problem_from_workload(small)
    q.grid.workspace = 256  # any non-NULL pointer: refused before it is used
    q.grid.workspace_bytes = 1 << 20
    with pytest.raises(btrt.BtrtError) as e:
        btrt.lib()  # loaded
        from ctypes import byref, c_double, c_int64
        out = np.empty((32, 32))
        phi0 = np.ascontiguousarray(small.phi0())
        rc = btrt.lib().btrt_solve_static(byref(q.grid), *q.args()[1:], btrt._dptr(phi0), 0.0, 10, btrt._dptr(out),
                                          byref(c_int64()), byref(c_double()))
        btrt._check(rc, "btrt_solve_static")
    assert e.value.code == btrt.E_INVAL and "workspace must be NULL" in str(e.value)
