"""A general D(phi) = (g phi + e |phi|^s) I (Eq. (1), Eq. (7)) through the C ABI.

* FP64 parity with the oracle (1e-12 normwise on phi and every population) on a periodic and a
  walled problem, ragged sizes included;
* every launch shape gives the same bits; D = (1 phi + 0) I gives the bits of D = phi I;
* FP32 storage within a stated bound of the oracle;
* from the HIP path: D = (phi + beta phi^3 / 3) I with A0 and D = phi I with A0 (1 + beta phi^2)
  converge to each other at second order (the same equation), at sizes past the oracle's reach.
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


def bump(n, m=None):
    m = n if m is None else m
    x, y = np.arange(n) + 0.5, np.arange(m) + 0.5
    X, Y = np.meshgrid(x, y)
    return 0.4 + 0.5 * np.exp(-((X - n / 2) ** 2 + (Y - m / 2) ** 2) / (2 * (min(n, m) / 8) ** 2))


def periodic_case(n=77, m=53):
    w = W.Workload(f"dterm_periodic_{n}x{m}", n, m, 150, A0=(0.06, 0.01, 0.03), flux_a=(0.03, -0.02),
                   flux_b=(0.02, 0.01), dterm=(0.9, 0.25, 2.5))
    return w, bump(n, m)


def walls_case(n=70, m=66):
    w = W.Workload(f"dterm_walls_{n}x{m}", n, m, 130, A0=(0.05, 0.0, 0.04), beta=0.5, flux_a=(0.02, 0.01),
                   dterm=(1.0, 0.3, 3.0), source=("sin", 1e-3, 1, 1), bc_type=(1, 1, 1, 1),
                   bc_value=(0.4, 0.5, 0.45, 0.6))
    return w, bump(n, m)


CASES = [periodic_case(), walls_case()]


class _W:
    """The workload with the given initial field (the oracle helpers call w.phi0())."""

    def __init__(self, w, phi0):
        self.__dict__.update(w.__dict__)
        self._phi0 = phi0

    def phi0(self):
        return self._phi0


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0].name)
def test_fp64_parity_with_oracle(case):
    w, phi0 = case
    say(f"[gpu] dterm parity {w.name} steps={w.steps}")
    with btrt.Solver(btrt.problem_from_workload(w), phi0) as s:
        s.step(w.steps)
        phi, f = s.field(), s.populations()
    o = run_oracle(_W(w, phi0))
    e_phi, e_f = normwise(phi, o.phi()), normwise(f, o.f)
    say(f"    normwise phi {e_phi:.3e}  f {e_f:.3e}")
    assert e_phi <= 1e-12 and e_f <= 1e-12


SHAPES = [(1, 4, 0, 0), (1, 16, 0, 0), (2, 0, 0, 1), (2, 8, 1, 0), (3, 16, 4, 0), (4, 8, 1, 0), (4, 32, 4, 0), (5, 16, 4, 0), (6, 32, 1, 0), (7, 16, 1, 0)]


@pytest.mark.parametrize("precision", [btrt.F64, btrt.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0].name)
def test_launch_shapes_bitwise(case, precision):
    w, phi0 = case
    steps = 33
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision), phi0) as ref:
        ref.set_fusion(1).step(steps)
        want = ref.populations()
    for shape in SHAPES:
        with btrt.Solver(btrt.problem_from_workload(w, precision=precision), phi0) as s:
            s.set_launch(*shape).step(steps)
            assert np.array_equal(s.populations(), want), shape


def test_linear_d_is_phi_i_bitwise():
    w, phi0 = walls_case()
    w.dterm = None
    for shape in [(1, 4, 0, 0), (4, 8, 1, 0)]:
        with btrt.Solver(btrt.problem_from_workload(w), phi0) as a:
            a.set_launch(*shape).step(40)
            fa = a.populations()
        w2, _ = walls_case()
        w2.dterm = (1.0, 0.0, 1.0)
        with btrt.Solver(btrt.problem_from_workload(w2), phi0) as b:
            b.set_launch(*shape).step(40)
            fb = b.populations()
        assert np.array_equal(fa, fb), shape


def test_fp32_bound():
    w, phi0 = periodic_case()
    with btrt.Solver(btrt.problem_from_workload(w, precision=btrt.F32), phi0) as s:
        s.step(w.steps)
        phi = s.field()
    ref = run_oracle(_W(w, phi0)).phi()
    e = normwise(phi, ref)
    say(f"    dterm f32 normwise {e:.3e}")
    assert e <= 5e-5


def test_equivalent_equations_converge_on_the_gpu():
    diffs = []
    for n in (64, 128, 256):
        steps = 100 * (n // 32) ** 2
        phi0 = bump(n)
        common = dict(A0=(0.06, 0.01, 0.03), flux_a=(0.02 * 32 / n, -0.01 * 32 / n))
        wa = W.Workload("a", n, n, steps, beta=2.0, **common)
        wb = W.Workload("b", n, n, steps, dterm=(1.0, 2.0 / 3.0, 3.0), **common)
        out = []
        for w in (wa, wb):
            with btrt.Solver(btrt.problem_from_workload(w), phi0) as s:
                s.step(steps)
                out.append(s.field())
        diffs.append(np.max(np.abs(out[0] - out[1])) / 0.5)
    orders = [np.log2(diffs[i] / diffs[i + 1]) for i in range(2)]
    say(f"    A(phi) vs D(phi): {diffs} orders {orders}")
    assert all(1.85 <= q <= 2.15 for q in orders), (diffs, orders)
