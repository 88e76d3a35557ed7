"""The largest grids one MI355X holds, run through the C ABI: 46336 x 46336 nodes (the largest square
whose padded planes stay below 2^31 elements, the library's index limit) in FP32 storage (~206 GB)
and in FP16 deviations (~129 GB), and 32768 x 32768 in FP64 (~189 GB).

phi0 repeats a seeded 64 x 64 pattern, so on a periodic grid the exact solution repeats too: every
64 x 64 tile of the GPU field must equal the first one bit for bit (which checks the indexing over
the whole grid), and the first tile must match the FP64 oracle run on the 64 x 64 pattern, within
the storage format's bound. Six steps run in one six-step walker launch and one more in the one-step
kernel; mass is conserved."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W
from tests._cases import normwise, oracle_problem

pytestmark = pytest.mark.gpu

P = 64


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pattern():
    x = (np.arange(P) + 0.5) / P
    X, Y = np.meshgrid(x, x)
    return 0.5 + 0.25 * np.sin(2 * np.pi * X) * np.cos(4 * np.pi * Y) + 0.15 * np.cos(2 * np.pi * (X + 2 * Y))


def workload(n):
    return W.Workload(f"max_{n}", n, n, 7, flux_b=(0.025, 0.025), flux_a=(0.01, -0.01), A0=(0.01, 0.0, 0.005),
                      beta=1.0)


@pytest.mark.parametrize("n,precision,bound", [(46336, btrt.F32, 5e-5), (46336, btrt.F16DEV, 1e-4),
                                               (32768, btrt.F64, 1e-12)], ids=["f32_46336", "f16dev_46336", "f64_32768"])
def test_largest_grid(n, precision, bound):
    w = workload(n)
    say(f"[gpu] max size {n}x{n} precision {precision}")
    p = btrt.problem_from_workload(w, precision=precision)
    assert p.validate().pitch == n
    phi0 = np.tile(pattern(), (n // P, n // P))
    m0 = float(np.sum(phi0))
    with btrt.Solver(p, phi0) as s:
        del phi0
        s.set_launch(6, 64, 1, 0).step(6)
        s.set_launch(1, 4, 0, 0).step(1)
        phi = s.field()
    say(f"    field read; checking tiles")
    first = phi[:P, :P].copy()
    for ty in (0, 1, n // P // 2, n // P - 1):
        for tx in (0, 1, n // P // 3, n // P - 1):
            assert np.array_equal(phi[ty * P:(ty + 1) * P, tx * P:(tx + 1) * P], first), (ty, tx)
    # Every tile along one band and one column of tiles, and the whole grid folded onto one tile.
    assert np.array_equal(phi[:P].reshape(P, n // P, P).transpose(1, 0, 2), np.broadcast_to(first, (n // P, P, P)))
    assert np.array_equal(phi[:, :P].reshape(n // P, P, P), np.broadcast_to(first, (n // P, P, P)))
    m1 = float(np.sum(phi, dtype=np.float64))
    del phi
    small = W.Workload("max_tile", P, P, 7, flux_b=w.flux_b, flux_a=w.flux_a, A0=w.A0, beta=w.beta)
    o = O.Oracle(oracle_problem(small), pattern(), nthreads=0).step(7)
    e = normwise(first, o.phi())
    say(f"    first tile vs oracle normwise {e:.3e}; mass drift {abs(m1 - m0) / m0:.2e}")
    assert e <= bound
    assert abs(m1 - m0) <= (1e-9 if precision == btrt.F64 else 1e-4) * m0
