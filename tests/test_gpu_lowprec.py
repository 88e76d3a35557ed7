"""16-bit scaled-deviation storage (BTRT_F16DEV, BTRT_BF16DEV) through the C ABI.

The populations are stored as 16-bit values of s * (f+ - f_eq(phi)) with phi kept in FP32 and
s a power of two fixed at set-up; the arithmetic is FP32. Checked here:
  * k steps per launch give the bits of k single steps, for every boundary combination
    (the fused kernel applies the same 16-bit round trip to the levels it keeps on chip);
  * splitting a run into several calls does not change a bit;
  * the initial populations are f_eq(phi0) (Section 4) within the rounding of the stored
    deviations, element by element;
  * the error against the FP64 oracle stays within stated bounds (normwise max and L2), which
    were measured on these inputs and carry a margin;
  * residual (Eq. (64)) and solve work on the 16-bit state;
  * batches and the server refuse these formats with BTRT_E_INVAL.
"""
import sys

import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W
from tests._cases import normwise, run_oracle
from tests.test_gpu_parity import CASES, custom

pytestmark = pytest.mark.gpu

FORMATS = [btrt.F16DEV, btrt.BF16DEV]
FMT_ID = {btrt.F16DEV: "f16dev", btrt.BF16DEV: "bf16dev"}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver(w, precision):
    return btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0())


@pytest.mark.parametrize("k", [2, 4, 6, 7])
@pytest.mark.parametrize("precision", FORMATS, ids=lambda p: FMT_ID[p])
@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_fused_launch_is_bitwise_identical(w, precision, k):
    steps = min(w.steps, 151) | 1
    say(f"[gpu] {FMT_ID[precision]} fused {k} vs single {w.name} {w.nx}x{w.ny} steps={steps}")
    with solver(w, precision) as a, solver(w, precision) as b:
        a.set_fusion(1).step(steps)
        b.set_fusion(k).step(steps)
        assert np.array_equal(a.populations(), b.populations())
        assert np.array_equal(a.field(), b.field())


@pytest.mark.parametrize("precision", FORMATS, ids=lambda p: FMT_ID[p])
def test_step_split_is_bitwise_invariant(precision):
    w = W.c2().scaled(77, 51, 0)
    say(f"[gpu] {FMT_ID[precision]} step split")
    with solver(w, precision) as a, solver(w, precision) as b:
        a.step(257)
        for k in (1, 0, 100, 56, 100):
            b.step(k)
        assert np.array_equal(a.populations(), b.populations())


# Unit roundoff of the 16-bit codes (round to nearest even): 2^-11 for binary16, 2^-8 for bfloat16.
UNIT = {btrt.F16DEV: 2.0 ** -11, btrt.BF16DEV: 2.0 ** -8}
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def initial_bound(feq, precision):
    """Element-wise bound on |f(0) - f_eq(phi0)| for the 16-bit formats on a periodic grid.

    f(0) at node y in direction i is pulled from x = y - c_i, which stores
    q(s (f_eq,i(phi0(y)) - f_eq,i(phi0(x)))) against its own equilibrium; the code rounds that
    difference to the format's unit roundoff u, plus a few FP32 roundings of the equilibrium
    itself and the subnormal spacing of binary16 (2^-24 / s, below 1e-11 of max|phi| here)."""
    d = np.empty_like(feq)
    for i in range(9):
        d[i] = feq[i] - np.roll(feq[i], shift=(CY[i], CX[i]), axis=(0, 1))
    return UNIT[precision] * np.abs(d) + 8 * 2.0 ** -24 * np.max(np.abs(feq))


@pytest.mark.parametrize("precision", FORMATS, ids=lambda p: FMT_ID[p])
@pytest.mark.parametrize("w", [W.c1(1.0), W.c3().scaled(96, 80, 0), custom("rough_periodic", 70, 45, 0)],
                         ids=lambda w: w.name)
def test_initial_populations_are_equilibrium(w, precision):
    say(f"[gpu] {FMT_ID[precision]} initial state {w.name}")
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision, check_interval=10), w.phi0()) as s:
        s.step(0)
        f = s.populations()
        r0 = s.residual()  # Eq. (64): phi(0) against phi0
    feq = run_oracle(w, steps=0).f  # f(0) = f_eq(phi0) (Section 4 initialisation)
    bound = initial_bound(feq, precision)
    err = np.abs(f - feq)
    say(f"    max err {err.max():.3e}  max err/bound {np.max(err / bound):.3f}  residual {r0:.3e}")
    assert np.all(err <= bound)
    assert r0 <= np.sum(bound) / np.sum(np.abs(w.phi0()))


# Stated bounds (normwise max and L2 of phi against the FP64 oracle), measured with margin.
ERROR_CASES = [
    (W.c1(1.0), {btrt.F16DEV: 1e-4, btrt.BF16DEV: 1e-3}),
    (W.c2().scaled(131, 97, 600), {btrt.F16DEV: 1e-4, btrt.BF16DEV: 1e-3}),
    (W.c3().scaled(193, 150, 300), {btrt.F16DEV: 1e-4, btrt.BF16DEV: 1e-3}),
    (custom("mixed_bc_xper_ywall", 70, 45, 400, bc_type=(0, 0, 1, 1), bc_value=(0, 0, 0.3, 0.8),
            source=("sin", 0.002, 2, 1)), {btrt.F16DEV: 1e-4, btrt.BF16DEV: 1e-3}),
]


@pytest.mark.parametrize("precision", FORMATS, ids=lambda p: FMT_ID[p])
@pytest.mark.parametrize("w,bounds", ERROR_CASES, ids=lambda v: getattr(v, "name", ""))
def test_error_against_fp64_oracle(w, bounds, precision):
    say(f"[gpu] {FMT_ID[precision]} error {w.name} {w.nx}x{w.ny} steps={w.steps}")
    with solver(w, precision) as s:
        s.step(w.steps)
        phi = s.field()
    ref = run_oracle(w).phi()
    e_max = normwise(phi, ref)
    e_l2 = float(np.sqrt(np.sum((phi - ref) ** 2) / np.sum(ref ** 2)))
    say(f"    {FMT_ID[precision]} normwise max {e_max:.3e}  l2 {e_l2:.3e}  bound {bounds[precision]:.0e}")
    assert e_max <= bounds[precision] and e_l2 <= bounds[precision]


@pytest.mark.parametrize("precision", FORMATS, ids=lambda p: FMT_ID[p])
def test_residual_and_solve(precision):
    w = W.c1(1.0)
    say(f"[gpu] {FMT_ID[precision]} residual / solve")
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision, check_interval=200), w.phi0()) as s:
        steps, res = s.solve(1e-30, 600)
        assert steps == 600 and res > 0
        assert s.info().step == 600
        assert s.info().bytes_per_node_launch == 18 * 2 + 2 * 4


@pytest.mark.parametrize("precision", FORMATS, ids=lambda p: FMT_ID[p])
def test_batch_and_server_refuse_deviation_formats(precision):
    w = W.c1(1.0)
    p = btrt.problem_from_workload(w, precision=precision)
    with pytest.raises(btrt.BtrtError) as e:
        btrt.Batch([(p, w.phi0())])
    assert e.value.code == btrt.E_INVAL
    with pytest.raises(btrt.BtrtError) as e:
        btrt.Server(precision=precision)
    assert e.value.code == btrt.E_INVAL
