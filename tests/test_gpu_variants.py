"""Method variants through the C ABI: a space-dependent diffusion tensor A0(x) and a source that
grows in time (Eqs. (73)-(76), Scheme 2 of Remark III).

* FP64 parity with the oracle (1e-12 normwise, phi and every population) on the Table 6 problem
  at several alpha and sizes (ragged included), and on a variant with Dirichlet walls and a
  separable source, both with a growing source;
* every launch shape gives the same bits (the per-step source factors are computed on the host,
  so fused launches see the same values as single steps);
* FP32 and FP16-deviation storage within stated bounds of the oracle;
* the Table 6 errors (Eq. (63)) computed from the HIP path's field;
* batches and the server refuse these variants with BTRT_E_INVAL.
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


def walls_variant(n=45, alpha=1e-3, steps=240):
    w = W.c6(alpha, n)
    w.name = f"c6_walls_{n}"
    w.steps = steps
    w.bc_type = (1, 1, 1, 1)
    w.bc_value = (0.1, 0.2, 0.3, 0.4)
    c = (np.arange(n) + 0.5) / n
    w.source = ("field", 2e-3 * np.outer(np.sin(np.pi * c), np.sin(2 * np.pi * c)), 0.004)  # rows: y
    return w


CASES = [W.c6(1e-2, 50), W.c6(1e-4, 64), W.c6(1e-3, 77, t_end=2.0), walls_variant()]


def exact_c6(w, steps):
    e = w.extra
    t = steps * e["dt"]
    c = (np.arange(w.nx) + 0.5) * e["dx"]
    X, Y = np.meshgrid(c, c)
    return np.exp(e["lambda"] * t) * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_fp64_parity_with_oracle(w):
    say(f"[gpu] variant parity {w.name} {w.nx}x{w.ny} steps={w.steps}")
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        s.step(w.steps)
        phi, f = s.field(), s.populations()
        assert s.info().k1_per_node == 1
    o = run_oracle(w)
    e_phi, e_f = normwise(phi, o.phi()), normwise(f, o.f)
    say(f"    normwise phi {e_phi:.3e}  f {e_f:.3e}")
    assert e_phi <= 1e-12 and e_f <= 1e-12


SHAPES = [(1, 4, 0, 0), (1, 16, 0, 0), (2, 0, 0, 1), (2, 8, 1, 0), (3, 16, 4, 0), (4, 8, 1, 0), (4, 32, 4, 0), (5, 16, 4, 0), (6, 32, 1, 0), (7, 16, 1, 0)]


@pytest.mark.parametrize("precision", [btrt.F64, btrt.F32, btrt.F16DEV], ids=["f64", "f32", "f16dev"])
@pytest.mark.parametrize("w", [CASES[0], CASES[3]], ids=lambda w: w.name)
def test_launch_shapes_bitwise(w, precision):
    steps = 31
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0()) as ref:
        ref.set_fusion(1).step(steps)
        want = ref.populations()
    for shape in SHAPES:
        with btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0()) as s:
            s.set_launch(*shape).step(steps)
            assert np.array_equal(s.populations(), want), shape


@pytest.mark.parametrize("precision,bound", [(btrt.F32, 5e-5), (btrt.F16DEV, 1e-4)], ids=["f32", "f16dev"])
def test_reduced_precision_bounds(precision, bound):
    w = W.c6(1e-3, 64, t_end=2.0)
    with btrt.Solver(btrt.problem_from_workload(w, precision=precision), w.phi0()) as s:
        s.step(w.steps)
        phi = s.field()
    ref = run_oracle(w).phi()
    e_max = normwise(phi, ref)
    e_l2 = float(np.sqrt(np.sum((phi - ref) ** 2) / np.sum(ref ** 2)))
    say(f"    variant {precision}: normwise max {e_max:.3e}  l2 {e_l2:.3e}")
    assert e_max <= bound and e_l2 <= bound


@pytest.mark.parametrize("alpha,n,printed", [(1e-4, 200, 1.7601e-4), (1e-6, 200, 1.7660e-4), (1e-4, 400, 4.2156e-5),
                                             (1e-6, 400, 4.1732e-5)])
def test_table6_errors_from_the_gpu(alpha, n, printed):
    w = W.c6(alpha, n)
    say(f"[gpu] Table 6 alpha={alpha} N={n} steps={w.steps}")
    with btrt.Solver(btrt.problem_from_workload(w), w.phi0()) as s:
        s.step(w.steps)
        phi = s.field()
    gre = O.gre(phi, exact_c6(w, w.steps))
    say(f"    GRE {gre:.4e} printed {printed:.4e}")
    assert gre == pytest.approx(printed, rel=0.15)


def test_batch_and_server_refuse_variants():
    w = W.c6(1e-3, 32)
    p = btrt.problem_from_workload(w, precision=btrt.F32)
    with pytest.raises(btrt.BtrtError) as e:
        btrt.Batch([(p, w.phi0())])
    assert e.value.code == btrt.E_INVAL
    with btrt.Server(precision=btrt.F32, memory_bytes=1 << 26) as srv:
        with pytest.raises(btrt.BtrtError) as e:
            srv.submit(p, w.phi0(), 1e-6, 100)
        assert e.value.code == btrt.E_INVAL
