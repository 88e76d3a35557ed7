"""Launch shapes on states larger than the 256 MiB Infinity Cache, where the one-step and two-step
tile kernels (single grids and batches) store non-temporally and the strip walkers do not.

Non-temporal stores change where the written lines are cached, not the values: every shape must
still give the bits of every other, on a single FP32 grid of 4096 x 1024 nodes (335 MB of state)
and on a batch of four FP32 instances of 1536^2 (755 MB), against the same instances stepped
alone (whose states fit the cache, so their kernels store normally).
"""
import dataclasses
import sys

import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_single_grid_shapes_agree_beyond_the_cache():
    w = W.c3().scaled(4096, 1024, 0)
    steps = 9
    say(f"[gpu] large state {w.nx}x{w.ny} FP32, {steps} steps per shape")
    out = {}
    for shape in [(1, 4, 0, 0), (1, 16, 0, 0), (2, 0, 0, 1), (4, 32, 4, 0), (7, 64, 1, 0)]:
        with btrt.Solver(btrt.problem_from_workload(w, precision=btrt.F32), w.phi0(), torch_memory=True) as s:
            s.set_launch(*shape).step(steps)
            out[shape] = (s.field(), s.populations())
    ref_phi, ref_f = out[(1, 4, 0, 0)]
    for shape, (phi, f) in out.items():
        assert np.array_equal(phi, ref_phi), shape
        assert np.array_equal(f, ref_f), shape


def test_batch_beyond_the_cache_equals_each_instance_alone():
    ws = [dataclasses.replace(W.c3().scaled(1536, 1536, 0), seed=100 + k) for k in range(4)]
    probs = [(btrt.problem_from_workload(w, precision=btrt.F32), w.phi0()) for w in ws]
    steps = 7
    for cfg in [(1, 0, 0), (2, 0, 0)]:
        say(f"[gpu] batch of 4 x 1536^2 FP32, config {cfg}, {steps} steps")
        with btrt.Batch(probs) as b:
            b.set_config(*cfg).step(steps)
            got = [b.field(i) for i in range(b.n)]
        for i, (p, ph) in enumerate(probs):
            with btrt.Solver(btrt.problem_from_workload(ws[i], precision=btrt.F32), ph) as s:
                s.set_fusion(1).step(steps)
                assert np.array_equal(got[i], s.field()), (cfg, i)
