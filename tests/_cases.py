"""Turns a seeded workload into the oracle's problem (test side only).

The oracle derives everything it needs (k2 of Eq. (62), the source field) with its own
formulas; nothing here comes from the HIP library.
"""
import numpy as np

from oracle import oracle as O


def oracle_problem(w) -> "O.Problem":
    if isinstance(w.k2, str):
        assert w.k2 == "hbb"
        k2 = (O.k2_hbb(O.k1_isotropic(w.A0[0])),) * 4
    elif np.isscalar(w.k2):
        k2 = (float(w.k2),) * 4
    else:
        k2 = tuple(w.k2)
    return O.Problem(w.nx, w.ny, flux_a=w.flux_a, flux_b=w.flux_b, A0=w.A0, beta=w.beta, k0=w.k0, K2=k2,
                     bc_type=w.bc_type, bc_value=w.bc_value)


def oracle_source(w):
    if w.source is None:
        return None
    kind, amp, kx, ky = w.source
    assert kind == "sin"
    return O.source_sin(w.nx, w.ny, amp, kx, ky)


def run_oracle(w, steps=None, nthreads=0) -> "O.Oracle":
    o = O.Oracle(oracle_problem(w), w.phi0(), source=oracle_source(w), nthreads=nthreads)
    o.step(w.steps if steps is None else steps)
    return o


def normwise(a, ref):
    """max |a - ref| / max |ref| (the normwise relative error used for parity)."""
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))
