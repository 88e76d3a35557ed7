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
                     bc_type=w.bc_type, bc_value=w.bc_value, A0_field=getattr(w, "A0_field", None),
                     flux_c=w.flux_c, flux_q=w.flux_q, src_r=w.src_r, src_p=w.src_p, dterm=w.dterm)


def oracle_source(w):
    """The time-independent part of the source (the whole source unless it grows in time)."""
    if w.source is None:
        return None
    if w.source[0] == "field":
        return np.ascontiguousarray(w.source[1], dtype=np.float64)
    kind, amp, kx, ky = w.source
    assert kind == "sin"
    return O.source_sin(w.nx, w.ny, amp, kx, ky)


def source_growth(w) -> float:
    return float(w.source[2]) if w.source is not None and w.source[0] == "field" else 0.0


def advance(o, w, n):
    """n oracle steps; a source exp(g t) S1(x) is evaluated at every step t, with S(t-1) for
    Scheme 2 (Remark III) and S(-1) := S(0); Dirichlet values that change in time are taken
    from the workload's schedule at every step."""
    g = source_growth(w)
    if g == 0.0 and w.walls is None:
        o.step(n)
        return o
    base = o.source
    links = None
    if w.walls is not None:
        links = getattr(o, "_wall_links", None)
        if links is None:
            links = o._wall_links = O.WallLinks(w.nx, w.ny, w.bc_type)
    for _ in range(n):
        t = o.t
        S = S_prev = None
        if g != 0.0:
            S = np.exp(g * t) * base
            S_prev = np.exp(g * (t - 1)) * base if t > 0 else S
        wall = links(w.walls(t)) if links is not None else None
        o.step(1, S=S, S_prev=S_prev, wall=wall)
    return o


def run_oracle(w, steps=None, nthreads=0) -> "O.Oracle":
    o = O.Oracle(oracle_problem(w), w.phi0(), source=oracle_source(w), nthreads=nthreads)
    return advance(o, w, w.steps if steps is None else steps)


def normwise(a, ref):
    """max |a - ref| / max |ref| (the normwise relative error used for parity)."""
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def oracle3_problem(w):
    """The oracle's D3Q19 problem for a workloads.Workload3."""
    from oracle import oracle3 as O3

    if isinstance(w.k2, str):
        assert w.k2 == "hbb"
        k2 = (O.k2_hbb(O.k1_isotropic(w.A0[0])),) * 9
    elif np.isscalar(w.k2):
        k2 = (float(w.k2),) * 9
    else:
        k2 = tuple(w.k2)
    return O3.Problem3(w.nx, w.ny, w.nz, flux_a=w.flux_a, flux_b=w.flux_b, A0=w.A0, beta=w.beta, k0=w.k0, K2=k2,
                       bc_type=w.bc_type, bc_value=w.bc_value)


def run_oracle3(w, steps=None, nthreads=0):
    from oracle import oracle3 as O3

    o = O3.Oracle3(oracle3_problem(w), w.phi0(), source=w.source, nthreads=nthreads)
    return o.step(w.steps if steps is None else steps)
