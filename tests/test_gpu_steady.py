"""Runs to a steady state: btrt_solve against the oracle with the same checks.

The anisotropic workload with Dirichlet walls and the separable source (A = [[0.02, 0.008],
[0.008, 0.01]], B = (0.02 phi, 0), S = sin(pi x / L) sin(pi y / L), phi0 ~ U[0, 1)) on small grids
(40 x 28, ragged against every strip and tile; 64 x 64) is solved until the Eq. (64) residual,
checked every 1000 steps, is at most 1e-10. The oracle takes the same checks (relative L1 change
of phi since the previous check, phi0 before the first): both stop at the same step, and the
state at that step agrees to 1e-12 normwise; the automatic launch shape and four- and seven-step
walkers give the same bits. The full 1024 x 1024 grid must reach the same tolerance within
100 000 steps (the step count is printed; the oracle is not run at that size).
"""
import sys

import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W
from tests._cases import advance, normwise, run_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-10
INTERVAL = 1000


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_solve(w, tol, cap):
    """Eq. (64) checks every INTERVAL oracle steps until the residual is at most tol."""
    o = run_oracle(w, 0)
    snap = w.phi0()
    steps, res = 0, np.inf
    while steps < cap:
        advance(o, w, INTERVAL)
        steps += INTERVAL
        phi = o.phi().copy()
        res = float(np.sum(np.abs(phi - snap)) / np.sum(np.abs(phi)))
        snap = phi
        if res <= tol:
            break
    return steps, res, o.phi().copy(), o.f.copy()


def gpu_solve(w, shape, tol, cap):
    prob = btrt.problem_from_workload(w, check_interval=INTERVAL)
    with btrt.Solver(prob, w.phi0()) as s:
        if shape is not None:
            s.set_launch(*shape)
        steps, res = s.solve(tol, cap)
        assert s.info().step == steps
        return steps, res, s.field(), s.populations()


@pytest.mark.parametrize("nx,ny", [(40, 28), (64, 64)])
def test_steady_state_matches_the_oracle(nx, ny):
    w = W.c2().scaled(nx, ny, 0)
    cap = 100 * INTERVAL
    o_steps, o_res, o_phi, o_f = oracle_solve(w, TOL, cap)
    assert o_res <= TOL and o_steps < cap
    first = None
    for shape in (None, (4, 16, 1, 0), (7, 8, 1, 0)):
        say(f"[gpu] steady {nx}x{ny} shape={shape} (oracle: {o_steps} steps, residual {o_res:.2e})")
        steps, res, phi, f = gpu_solve(w, shape, TOL, cap)
        assert steps == o_steps, (steps, o_steps)
        assert res <= TOL
        assert res == pytest.approx(o_res, rel=1e-2, abs=1e-15)
        assert normwise(phi, o_phi) <= 1e-12
        assert normwise(f, o_f) <= 1e-12
        if first is None:
            first = (phi, f)
        else:
            assert np.array_equal(phi, first[0]) and np.array_equal(f, first[1]), shape


def test_full_size_reaches_the_tolerance():
    # Advection at u = 0.02 has flushed the initial data after ~L/u = 51 200 steps; the first
    # check at or below 1e-10 comes soon after (63 000 steps on the measured runs).
    w = W.c2()
    prob = btrt.problem_from_workload(w, check_interval=INTERVAL)
    with btrt.Solver(prob, w.phi0()) as s:
        steps, res = s.solve(TOL, 100 * INTERVAL)
        say(f"[gpu] c2 1024^2: {steps} steps, residual {res:.3e}")
        assert s.info().step == steps
        assert np.isfinite(res) and res <= TOL and steps < 100 * INTERVAL
        assert np.all(np.isfinite(s.field()))
