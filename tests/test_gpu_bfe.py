"""The Burgers-Fisher variant through the C ABI (Eqs. (67)-(69)): the general node model with a
power-law flux, a phi-dependent source under Scheme 2 and Dirichlet values that change along the
walls and in time (btrt_set_walls).

* FP64 parity with the oracle (1e-12 normwise on phi and every population), on square and
  ragged grids, with walls on all sides and with one direction periodic, read mid-run as well;
* every launch shape gives the same bits (the wall table is indexed by the step inside a fused
  launch, so a level that read the wrong entry would differ);
* a schedule holding the per-side constants reproduces a handle without one, bit for bit;
* a schedule set in two parts equals one set at once; steps past its end are refused and leave
  the state untouched; btrt_tune stays inside it;
* FP32 storage within a stated bound of the oracle; Tables 4 and 5 from the HIP path's field, to
  the printed digits (the walls taken where each link meets them);
* unequal walls that vary along every side, with a different value at each corner from each of
  the two sides (the corner links take their mean), in every launch shape;
* batches and the server refuse the general model.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W
from tests._cases import normwise, run_oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver(w, precision=btrt.F64, steps=None):
    s = btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0())
    s.set_walls(btrt.wall_schedule(w, 0, w.steps if steps is None else steps))
    return s


def half_periodic(n=20):
    w = W.bfe(n=n, alpha=0.05, t_end=0.6)
    w.name = f"bfe_periodic_x_{w.nx}"
    w.bc_type = (btrt.PERIODIC, btrt.PERIODIC, btrt.DIRICHLET, btrt.DIRICHLET)
    w.bc_value = (0.0, 0.0, 0.0, 0.0)
    return w


def ragged(n=21):
    w = W.bfe(n=n, alpha=0.01, a=1.0, t_end=0.5)
    w.name = f"bfe_ragged_{w.nx}"
    return w


CASES = [W.bfe(n=20, alpha=0.05, t_end=1.0), ragged(), half_periodic(), W.bfe(n=40, alpha=0.005, t_end=0.4)]


def exact(w, steps):
    e = w.extra
    c = e["x0"] + (np.arange(w.nx) + 0.5) * e["dx"]
    X, Y = np.meshgrid(c, c)
    return O.burgers_fisher(X, Y, steps * e["dt"], e["a"], e["alpha"], e["b"], e["delta"])


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_fp64_parity_with_oracle(w):
    say(f"[gpu] bfe parity {w.name} {w.nx}x{w.ny} steps={w.steps}")
    mid = w.steps // 3
    with solver(w) as s:
        s.step(mid)
        phi_mid = s.field()
        s.step(w.steps - mid)
        phi, f = s.field(), s.populations()
    o_mid = run_oracle(w, steps=mid)
    e_mid = normwise(phi_mid, o_mid.phi())
    o = run_oracle(w)
    e_phi, e_f = normwise(phi, o.phi()), normwise(f, o.f)
    say(f"    normwise phi(mid) {e_mid:.3e}  phi {e_phi:.3e}  f {e_f:.3e}")
    assert e_mid <= 1e-12 and e_phi <= 1e-12 and e_f <= 1e-12


SHAPES = [(1, 4, 0, 0), (1, 16, 0, 0), (2, 0, 0, 1), (2, 8, 1, 0), (3, 16, 4, 0), (4, 8, 1, 0), (4, 32, 4, 0),
          (4, 128, 1, 0), (5, 16, 4, 0), (6, 32, 1, 0), (7, 64, 1, 0)]


@pytest.mark.parametrize("precision", [btrt.F64, btrt.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("w", [CASES[1], CASES[2]], ids=lambda w: w.name)
def test_launch_shapes_bitwise(w, precision):
    steps = 37
    with solver(w, precision, steps) as ref:
        ref.set_fusion(1).step(steps)
        want = ref.populations()
    for shape in SHAPES:
        with solver(w, precision, steps) as s:
            s.set_launch(*shape).step(steps)
            assert np.array_equal(s.populations(), want), shape


@pytest.mark.parametrize("precision", [btrt.F64, btrt.F32], ids=["f64", "f32"])
def test_constant_schedule_equals_constant_walls(precision):
    # A problem without the power-law flux or the reaction, once with per-side constants and once
    # with a schedule that holds the same constants: the general kernels must give the same bits.
    nx, ny, steps = 70, 45, 29
    w = W.Workload("walls_const", nx, ny, steps, A0=(0.03, 0.004, 0.02), flux_a=(0.04, -0.03), flux_b=(0.02, 0.0),
                   bc_type=(1, 1, 1, 1), bc_value=(0.2, -0.1, 0.5, 0.3), seed=11)
    row = np.concatenate([np.full(2 * ny + 1, 0.2), np.full(2 * ny + 1, -0.1), np.full(2 * nx + 1, 0.5),
                          np.full(2 * nx + 1, 0.3)])
    for shape in [(1, 4, 0, 0), (2, 0, 0, 1), (4, 8, 1, 0), (3, 16, 4, 0)]:
        with btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0()) as a:
            a.set_launch(*shape).step(steps)
            fa = a.populations()
        with btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0()) as b:
            b.set_walls(np.tile(row, (steps, 1)))
            b.set_launch(*shape).step(steps)
            fb = b.populations()
        assert np.array_equal(fa, fb), shape


def test_schedule_in_parts_and_its_end():
    w = CASES[0]
    n1, n2 = 30, 41
    with solver(w, steps=n1 + n2) as ref:
        ref.set_launch(4, 8, 1, 0).step(n1 + n2)
        want = ref.populations()
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        s.set_launch(4, 8, 1, 0)
        s.set_walls(btrt.wall_schedule(w, 0, n1)).step(n1)
        before = s.populations()
        with pytest.raises(btrt.BtrtError) as e:
            s.step(1)  # past the end of the schedule
        assert e.value.code == btrt.E_INVAL
        assert s.info().step == n1 and np.array_equal(s.populations(), before)
        s.set_walls(btrt.wall_schedule(w, n1, n2)).step(n2)
        assert np.array_equal(s.populations(), want)
        # The tuner never steps past the schedule either.
        s.set_walls(btrt.wall_schedule(w, n1 + n2, 20))
        _, used = s.tune(1000)
        assert used <= 20 and s.info().step == n1 + n2 + used
        with pytest.raises(btrt.BtrtError):
            s.set_walls(np.full((3, 4 * (w.nx + w.ny) + 4), np.nan))
        with pytest.raises(btrt.BtrtError):
            s.set_walls(np.zeros((0, 4 * (w.nx + w.ny) + 4)))


def test_fp32_bound():
    w = W.bfe(n=20, alpha=0.05, t_end=1.0)
    with solver(w, btrt.F32) as s:
        s.step(w.steps)
        phi = s.field()
    ref = run_oracle(w).phi()
    e_max = normwise(phi, ref)
    e_l2 = float(np.sqrt(np.sum((phi - ref) ** 2) / np.sum(ref ** 2)))
    say(f"    bfe f32: normwise max {e_max:.3e}  l2 {e_l2:.3e}")
    assert e_max <= 2e-5 and e_l2 <= 2e-5


@pytest.mark.parametrize("a,alpha,printed", [(2.0, 0.05, 9.5559e-4), (1.0, 0.05, 5.0193e-4), (2.0, 0.1, 2.0497e-3)])
def test_tables_4_5_from_the_gpu(a, alpha, printed):
    w = W.bfe(n=40, alpha=alpha, a=a, t_end=1.0)
    with solver(w) as s:
        s.tune(60)
        s.step(w.steps - s.info().step)
        phi = s.field()
        err = s.error(exact(w, w.steps))
    gre = O.gre(phi, exact(w, w.steps))
    say(f"    GRE {gre:.4e} printed {printed:.4e}")
    assert err[0] == pytest.approx(gre, rel=1e-12)
    assert gre == pytest.approx(printed, rel=2e-4)


def rough_walls(w, seed=21):
    """A schedule of walls that differ along each side, between the sides and from step to step,
    so that every link of the boundary carries its own value; the two sides meeting at a corner
    disagree there."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(-0.5, 1.0, 4 * (w.nx + w.ny) + 4)
    return lambda k: base * (1.0 + 0.01 * np.sin(0.3 * k)) + 0.02 * k / max(w.steps, 1)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (0, 0, 1, 1), (1, 1, 0, 0)], ids=["walls", "x_periodic", "y_periodic"])
def test_rough_walls_every_link_and_corner(bc):
    w = W.Workload("rough_walls", 71, 45, 33, A0=(0.03, 0.006, 0.02), flux_a=(0.03, -0.02), flux_b=(0.02, 0.01),
                   beta=0.5, bc_type=bc, bc_value=tuple(0.1 * (q + 1) if t else 0.0 for q, t in enumerate(bc)),
                   k0=0.9, k2=(1.1, 0.95, 0.95, 1.2), seed=17)
    w.walls = rough_walls(w)
    say(f"[gpu] rough walls {w.nx}x{w.ny} bc={bc} steps={w.steps}")
    o = run_oracle(w)
    for shape in [(1, 4, 0, 0), (2, 0, 0, 1), (3, 16, 4, 0), (4, 8, 1, 0), (7, 64, 1, 0)]:
        with solver(w) as s:
            s.set_launch(*shape).step(w.steps)
            phi, f = s.field(), s.populations()
        e_phi, e_f = normwise(phi, o.phi()), normwise(f, o.f)
        say(f"    shape {shape}: normwise phi {e_phi:.3e}  f {e_f:.3e}")
        assert e_phi <= 1e-12 and e_f <= 1e-12, shape


def test_batch_and_server_refuse_the_general_model():
    w = W.bfe(n=10)
    p = btrt.problem_from_workload(w, precision=btrt.F32)
    with pytest.raises(btrt.BtrtError) as e:
        btrt.Batch([(p, w.phi0())])
    assert e.value.code == btrt.E_INVAL
    with btrt.Server(precision=btrt.F32, memory_bytes=1 << 26) as srv:
        with pytest.raises(btrt.BtrtError) as e:
            srv.submit(p, w.phi0(), 1e-6, 100)
        assert e.value.code == btrt.E_INVAL
    q = btrt.problem_from_workload(W.c1(), precision=btrt.F16DEV)
    with btrt.Solver(q, W.c1().phi0()) as s:
        with pytest.raises(btrt.BtrtError) as e:
            s.set_walls(np.zeros((2, 4 * 128 + 4)))
        assert e.value.code == btrt.E_INVAL
