"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64: normwise relative difference max|gpu - oracle| / max|oracle| <= 1e-12 for phi and for
every population (the tolerance the method's FP64 path is held to). Inputs come from the
seeded workloads; expected values from the oracle run on the same inputs.
"""
import sys

import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W
from tests._cases import normwise, oracle_problem, oracle_source, run_oracle
from oracle import oracle as O

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_run(w, precision=btrt.F64, steps=None, torch_memory=False):
    say(f"[gpu] {w.name} {w.nx}x{w.ny} steps={w.steps if steps is None else steps} prec={precision}")
    s = btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0(), torch_memory=torch_memory)
    s.step(w.steps if steps is None else steps)
    return s


def custom(name, nx, ny, steps, **kw):
    base = dict(flux_a=(0.03, -0.02), A0=(0.02, 0.006, 0.012), k0=0.9, k2=(0.8, 1.3, 0.5, 1.2), seed=11,
                phi0_kind="uniform")
    base.update(kw)
    return W.Workload(name, nx, ny, steps, **base)


CASES = [
    W.c1("hbb"),
    W.c1(1.0),
    W.c2().scaled(131, 97, 600),
    W.c3().scaled(193, 150, 300),
    custom("mixed_bc_xper_ywall", 70, 45, 400, bc_type=(0, 0, 1, 1), bc_value=(0, 0, 0.3, 0.8),
           source=("sin", 0.002, 2, 1)),
    custom("mixed_bc_xwall_yper", 45, 70, 400, bc_type=(1, 1, 0, 0), bc_value=(0.7, 0.2, 0, 0)),
    custom("all_walls_unequal_corners", 67, 33, 300, bc_type=(1, 1, 1, 1), bc_value=(0.1, 0.9, 0.4, 0.6),
           flux_b=(0.04, -0.03), beta=0.7),
    custom("tiny_1x1_periodic", 1, 1, 50),
    custom("tiny_1x7_walls", 1, 7, 80, bc_type=(1, 1, 1, 1), bc_value=(0.2, 0.5, 0.9, 0.1)),
    custom("tiny_5x1_mixed", 5, 1, 80, bc_type=(0, 0, 1, 1), bc_value=(0, 0, 0.3, 0.6)),
    custom("row_2x129_walls", 129, 2, 120, bc_type=(1, 1, 1, 1), bc_value=(0.5, 0.5, 0.5, 0.5)),
]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_fp64_parity_phi_and_populations(w):
    s = gpu_run(w)
    phi, f = s.field(), s.populations()
    s.close()
    o = run_oracle(w)
    e_phi = normwise(phi, o.phi())
    e_f = normwise(f, o.f)
    say(f"    normwise phi {e_phi:.3e}  f {e_f:.3e}")
    assert e_phi <= TOL64 and e_f <= TOL64


def test_fp64_parity_field_source():
    rng = np.random.default_rng(5)
    w = custom("field_source", 90, 70, 250, bc_type=(1, 1, 0, 0), bc_value=(0.25, 0.75, 0, 0))
    S = 1e-3 * rng.standard_normal((w.ny, w.nx))
    say(f"[gpu] field source {w.nx}x{w.ny}")
    p = btrt.Problem(w.nx, w.ny, flux_a=w.flux_a, A0=w.A0, source=S, bc_type=w.bc_type, bc_value=w.bc_value,
                     k0=w.k0, k2=w.k2)
    with btrt.Solver(p, w.phi0()) as s:
        s.step(w.steps)
        phi = s.field()
    o = O.Oracle(oracle_problem(w), w.phi0(), source=S)
    o.step(w.steps)
    assert normwise(phi, o.phi()) <= TOL64


@pytest.mark.parametrize("w,steps", [(W.c2(), 100), (W.c3(), 10)], ids=["c2_1024_100steps", "c3_4096_10steps"])
def test_fp64_parity_full_size_short(w, steps):
    # Full-size grids in the benchmark's launch configuration, for as many steps as the
    # oracle finishes in seconds.
    s = gpu_run(w, steps=steps)
    phi = s.field()
    s.close()
    o = run_oracle(w, steps=steps)
    e = normwise(phi, o.phi())
    say(f"    normwise phi {e:.3e}")
    assert e <= TOL64


def test_residual_and_error_norms():
    w = W.c2().scaled(100, 80, 0)
    say("[gpu] residual / error norms")
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        o = O.Oracle(oracle_problem(w), w.phi0(), source=oracle_source(w))
        snap = o.phi()
        for k in (300, 700):
            s.step(k)
            o.step(k)
            cur = o.phi()
            r_gpu = s.residual()
            r_orc = O.residual(cur, snap)  # Eq. (64) against the previous check
            snap = cur
            assert abs(r_gpu - r_orc) <= 1e-11 * r_orc, (r_gpu, r_orc)
        ref = W.c2().scaled(100, 80, 0).phi0() * 3.0 + 0.5
        gre, mx, l2 = s.error(ref)
        phi = o.phi()
        assert gre == pytest.approx(O.gre(phi, ref), rel=1e-12)
        assert mx == pytest.approx(np.max(np.abs(phi - ref)), rel=1e-12)
        assert l2 == pytest.approx(np.sqrt(np.sum((phi - ref) ** 2) / np.sum(ref ** 2)), rel=1e-12)


def test_residual_first_call_compares_to_phi0_and_solve_stops():
    w = W.c1(1.0)
    with btrt.Solver(btrt.problem_from_workload(w, check_interval=200), w.phi0()) as s:
        s.step(0)
        assert s.residual() == pytest.approx(0.0, abs=1e-15)  # phi(0) = sum f_eq(phi0) = phi0
        steps, res = s.solve(1e-30, 600)
        assert steps == 600 and res > 0
        assert s.info().step == 600


@pytest.mark.parametrize("w", [W.c3().scaled(130, 67, 120), W.c2().scaled(1400, 1300, 41)], ids=["small", "nt_stores"])
def test_torch_memory_and_stream_bitwise_identical(w):
    # The library's own allocation and a torch workspace on torch's stream give the same bits
    # (1400 x 1300 FP64 exceeds the 256 MB cache threshold and takes the non-temporal stores).
    a = gpu_run(w)
    b = gpu_run(w, torch_memory=True)
    pa, pb = a.field(), b.field()
    a.close()
    b.close()
    assert np.array_equal(pa, pb)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_fused_launch_is_bitwise_identical(w, k):
    # k steps per launch (strip walkers, intermediate levels in registers) must give the bits
    # of k single steps, for every boundary combination and a step count that ends with a
    # shorter launch.
    steps = min(w.steps, 151) | 1
    say(f"[gpu] fused {k} vs single {w.name} {w.nx}x{w.ny} steps={steps}")
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as a, \
            btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as b:
        a.set_fusion(1).step(steps)
        b.set_fusion(k).step(steps)
        assert np.array_equal(a.populations(), b.populations())
        assert np.array_equal(a.field(), b.field())


# Shapes around the walker's strip width (66 - 2k columns) and strip height (16 rows at these
# sizes), with every boundary combination.
WALK_SHAPES = [(57, 17), (58, 16), (59, 33), (60, 31), (62, 47), (116, 15), (125, 64), (1, 40), (130, 1), (3, 3)]
WALK_BCS = [(0, 0, 0, 0), (1, 1, 1, 1), (0, 0, 1, 1), (1, 1, 0, 0)]


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("shape", WALK_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_walker_strip_edges_bitwise(shape, k):
    nx, ny = shape
    for bc in WALK_BCS:
        w = custom(f"walk_{nx}x{ny}", nx, ny, 0, bc_type=bc, bc_value=(0.2, 0.7, 0.4, 0.9), flux_b=(0.04, -0.03),
                   beta=0.5, source=("sin", 0.003, 1, 2))
        steps = 3 * k + 1
        say(f"[gpu] walker k={k} {nx}x{ny} bc={bc} steps={steps}")
        with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as a, \
                btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as b:
            a.set_fusion(1).step(steps)
            b.set_fusion(k).step(steps)
            assert np.array_equal(a.populations(), b.populations()), bc


def test_fusion_outside_range_is_rejected():
    w = W.c1(1.0)
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        for k in (0, 8, -1):
            with pytest.raises(btrt.BtrtError) as e:
                s.set_fusion(k)
            assert e.value.code == btrt.E_INVAL


def test_step_split_is_bitwise_invariant():
    w = W.c2().scaled(77, 51, 0)
    p = btrt.problem_from_workload(w)
    with btrt.Solver(p, w.phi0()) as a, btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as b:
        a.step(257)
        for k in (1, 0, 100, 56, 100):
            b.step(k)
        assert np.array_equal(a.field(), b.field())


def test_unstable_run_is_reported():
    # LBGK rates (Table 1) at u = 0.5 lattice units diverge (Table 3: LBGK unstable at u0 = 2.5).
    tau = 0.8
    k1 = 1 / tau
    a = (tau - 0.5) / 3.0
    p = btrt.Problem(32, 32, flux_a=(0.5, 0.5), A0=(a, 0.0, a), k0=k1, k2=k1)
    phi0 = 1.0 + 0.01 * np.random.default_rng(0).random((32, 32))
    with btrt.Solver(p, phi0) as s:
        s.step(6000)
        with pytest.raises(btrt.BtrtError) as e:
            s.residual()
        assert e.value.code == btrt.E_UNSTABLE


# Stated FP32 bounds (normwise against the FP64 oracle), measured with margin.
FP32_CASES = [(W.c1(1.0), 5e-5), (W.c2().scaled(131, 97, 600), 5e-5), (W.c3().scaled(193, 150, 300), 5e-5)]


@pytest.mark.parametrize("w,bound", FP32_CASES, ids=lambda v: getattr(v, "name", str(v)))
def test_fp32_error_against_fp64_oracle(w, bound):
    s = gpu_run(w, precision=btrt.F32)
    phi = s.field()
    s.close()
    ref = run_oracle(w).phi()
    e_max = normwise(phi, ref)
    e_l2 = float(np.sqrt(np.sum((phi - ref) ** 2) / np.sum(ref ** 2)))
    say(f"    fp32 normwise max {e_max:.3e}  l2 {e_l2:.3e}")
    assert e_max <= bound and e_l2 <= bound
