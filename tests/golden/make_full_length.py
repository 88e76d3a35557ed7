"""Writes the full-length parity references by running the FP64 CPU oracle on the full workloads:
1024 x 1024 for 20000 steps and 4096 x 4096 for 5000 steps. Only the oracle is called.

Stored per workload:

* ``<workload>_full.json``: phi and all nine populations at seeded sample nodes (plus corners,
  edge midpoints and the centre), and whole-field norms;
* ``<workload>_full.npz``: phi on the strided subgrid of every 8th node in x and y (starting at
  node 0), and sums over each 64 x 64 block of nodes of phi, |phi|, phi^2 and of every population
  (block (by, bx) covers rows 64 by .. 64 by + 63 and columns 64 bx .. 64 bx + 63), each block
  summed in FP64 along rows, then over the block's rows in order.

    python tests/golden/make_full_length.py [c2|c3 ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_1902_09813_amd import workloads as W  # noqa: E402  (inputs only)
from tests._cases import run_oracle  # noqa: E402

STRIDE = 8
BLOCK = 64


def sample_nodes(nx, ny, seed=1234, count=256):
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, 0), (0, ny // 2), (nx - 1, ny // 2),
           (nx // 2, ny - 1), (nx // 2, ny // 2)}
    while len(pts) < count:
        pts.add((int(rng.integers(nx)), int(rng.integers(ny))))
    return sorted(pts)


def block_sums(a, block=BLOCK):
    """Sums of a (ny, nx) field over block x block tiles: shape (ny / block, nx / block)."""
    ny, nx = a.shape
    assert ny % block == 0 and nx % block == 0
    return a.reshape(ny // block, block, nx // block, block).sum(axis=3).sum(axis=1)


def make(name):
    w = {"c2": W.c2, "c3": W.c3}[name]()
    t = time.time()
    o = run_oracle(w)
    el = time.time() - t
    phi = o.phi()
    pts = sample_nodes(w.nx, w.ny)
    rec = {
        "workload": w.name,
        "nx": w.nx,
        "ny": w.ny,
        "steps": w.steps,
        "written_by": "tests/golden/make_full_length.py (FP64 CPU oracle only)",
        "oracle_seconds": round(el, 1),
        "nodes": pts,
        "phi": [repr(float(phi[y, x])) for x, y in pts],
        "f": [[repr(float(o.f[i, y, x])) for i in range(9)] for x, y in pts],
        "sum_phi": repr(float(np.sum(phi))),
        "sum_abs_phi": repr(float(np.sum(np.abs(phi)))),
        "max_abs_phi": repr(float(np.max(np.abs(phi)))),
        "sum_phi_sq": repr(float(np.sum(phi * phi))),
        "max_abs_f": repr(float(np.max(np.abs(o.f)))),
    }
    path = os.path.join(HERE, f"{w.name}_full.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=0)
    npz = os.path.join(HERE, f"{w.name}_full.npz")
    np.savez(npz, phi_sub=np.ascontiguousarray(phi[::STRIDE, ::STRIDE]), stride=np.int64(STRIDE),
             block=np.int64(BLOCK), block_phi=block_sums(phi), block_abs_phi=block_sums(np.abs(phi)),
             block_phi_sq=block_sums(phi * phi), block_f=np.stack([block_sums(o.f[i]) for i in range(9)]),
             max_abs_f_plane=np.array([np.max(np.abs(o.f[i])) for i in range(9)]))
    print(f"{name}: {w.nx}x{w.ny} x {w.steps} steps in {el:.0f} s -> {path}, {npz}", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c2", "c3"]:
        make(n)
