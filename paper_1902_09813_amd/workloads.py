"""Seeded synthetic workloads (problem parameters and initial fields), in lattice units.

This module holds inputs only: parameters and initial fields drawn from fixed seeds.
It contains none of the method's arithmetic, so the HIP path and the CPU oracle can
both take their inputs from here without sharing any computation.

Workloads (lattice units; the paper's problems are analytic, so no dataset is involved):

* ``c1``  64 x 64 periodic, A = 0.01 I, B = phi (0.05, 0.05), S = 0, phi0 a periodised
          Gaussian hill (sigma 6, centre at the box centre), 2000 steps. k2 from the
          bounce-back rule (Eq. (62)) or k2 = 1.
* ``c2``  1024 x 1024, Dirichlet phi_w = 0 on all sides, A = [[0.02, 0.008], [0.008, 0.01]],
          B = phi (0.02, 0), S = sin(pi x / L) sin(pi y / L), phi0 ~ U[0, 1) (seed 2),
          k0 = k2 = 1, 20000 steps.
* ``c3``  4096 x 4096 periodic, B = 0.025 phi^2 (1, 1), A(phi) = diag(0.01, 0.005)(1 + phi^2),
          S = 0, phi0 = sum of 16 Gaussians (seed 3; amplitude U[0, 1], sigma U[8, 64], centre
          U[0, 4096)^2, minimum-image distance), k0 = k2 = 1, 5000 steps.

* ``c4``  256 independent instances (seed 4): side N = round(exp(U[ln 32, ln 512])), k11, k22 ~
          U[0.005, 0.05], k12 ~ U[-0.5, 0.5] sqrt(k11 k22), u ~ U[-0.05, 0.05]^2; a seeded coin
          picks periodic or Dirichlet sides. Dirichlet: per-side phi_w ~ U[0, 1] and
          S = r0 sin(pi x/N) sin(pi y/N); periodic: S = r0 sin(2 pi x/N) sin(2 pi y/N) (zero
          mean); r0 ~ U[0, 1e-4]; phi0 ~ U[0, 1); k0 = k2 = 1; FP32 storage, 2000 steps.

* ``c5``  served requests (seed 5): Poisson arrival times at a given rate; side N log-uniform in
          [64, 2048]; coefficients, boundaries, sources and phi0 drawn as for ``c4``; half of
          the requests (seeded coin) use A(phi) = A0 (1 + phi^2); each runs until the Eq. (64)
          residual is <= 1e-8 or 50000 steps; FP32 storage.

* ``c6``  the variable diffusion tensor problem (Eqs. (73)-(76)): unit square, periodic,
          A(x) = diag(2 - sin(2 pi x) sin(2 pi y), 1) alpha, u = (0.1, 0.1), the source of
          Eq. (75) = exp((1 - 12 pi^2 alpha) t) S1(x), phi0 = sin(2 pi x) sin(2 pi y), k0 = k2 = 1;
          N x N cell-centred nodes, dt = dx (lattice speed 1) unless given. In lattice units the
          source is a field times exp(g n) at step n (g = lambda dt) and A0 is a per-node field.

* ``bfe``  the Burgers-Fisher equation (Eqs. (67)-(69)) on [-1, 2]^2 with N nodes per unit
          length (3N x 3N cell-centred nodes), lattice speed c (dt = dx / c), a = 2, b = 0.05,
          delta = 1.5 unless given: in lattice units B(phi) = (a / ((delta + 1) c)) |phi|^(delta+1)
          along x, A = alpha dt / dx^2 I, S(phi) = b dt phi (1 - |phi|^delta), k0 = 1, k2 from
          Eq. (62); phi0 and the Dirichlet values on all four walls from Eq. (68), the walls at
          time (k + 1) dt for the k-th step, sampled where the links meet them (every half
          lattice spacing along each side, corners included).

* ``d3``   three-dimensional (D3Q19) problems: ``d3_hill(n)`` an n^3 periodic box, anisotropic
          A0 = [[0.05, 0.01, 0.005], [0.01, 0.04, -0.008], [0.005, -0.008, 0.03]], B = phi u with
          u = (0.02, -0.01, 0.015) 16/n (diffusive scaling), phi0 the 3-D Gaussian of sigma n/6 at the
          box centre (periodic images |m| <= 1), k0 = k2 = 1; ``d3_nonlinear(nx, ny, nz)`` periodic,
          B = 0.025 phi^2 (1, 1, 1) + phi (0.01, 0, -0.01), A(phi) = diag(0.01, 0.008, 0.006)(1 + phi^2),
          phi0 a sum of 12 Gaussians (seed 7; amplitude U[0, 1], sigma U[0.06, 0.15] of the shortest side,
          centres uniform, minimum image), k0 = k2 = 1 (the 3-D counterpart of c3);
          ``d3_walls(nx, ny, nz)`` six Dirichlet faces phi_w = (0.2, 0.5, 0.3, 0.6, 0.4, 0.1),
          A0 full, beta = 0.5, B = phi (0.02, 0.01, -0.015) + 0.01 phi^2 (1, 0, 0), S = 1e-3 sin sin sin
          at cell centres, phi0 ~ U[0, 1) (seed 8), K2 rates 0.9 .. 1.3.

``scaled`` variants keep every parameter and shrink the grid (for parity at oracle-friendly
sizes; ragged sizes exercise partial tiles).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Callable, Optional, Tuple

import numpy as np

PERIODIC, DIRICHLET = 0, 1


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    steps: int
    flux_a: Tuple[float, float] = (0.0, 0.0)
    flux_b: Tuple[float, float] = (0.0, 0.0)
    A0: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    beta: float = 0.0
    source: Optional[tuple] = None          # None, ("sin", amp, kx, ky) or ("field", S1 (ny, nx), g):
    #                                         S(x, n) = exp(g n) S1(x) at step n
    A0_field: Optional[np.ndarray] = None   # (ny, nx, 3) per-node A0 = (a11, a12, a22), or None
    bc_type: Tuple[int, int, int, int] = (PERIODIC,) * 4
    bc_value: Tuple[float, float, float, float] = (0.0,) * 4
    k0: float = 1.0
    k2: object = 1.0                        # scalar, 4 entries, or "hbb" (Eq. (62))
    seed: int = 0
    phi0_kind: str = "uniform"
    extra: dict = field(default_factory=dict)
    flux_c: Tuple[float, float] = (0.0, 0.0)  # B(phi) gains c |phi|^q
    flux_q: float = 1.0
    src_r: float = 0.0                      # S gains r phi (1 - |phi|^p)
    src_p: float = 1.0
    walls: Optional[Callable[[int], np.ndarray]] = None  # k -> Dirichlet values of the k-th step
    #                                         at the points where links meet the sides, every half
    #                                         lattice spacing from corner to corner: x- (2 ny + 1),
    #                                         x+ (2 ny + 1), y- (2 nx + 1), y+ (2 nx + 1)
    dterm: Optional[Tuple[float, float, float]] = None  # D = (g phi + e |phi|^s) I; None: D = phi I

    def phi0(self) -> np.ndarray:
        return initial_field(self)

    def scaled(self, nx: int, ny: int, steps: Optional[int] = None) -> "Workload":
        return replace(self, nx=nx, ny=ny, steps=self.steps if steps is None else steps)


def c1(k2="hbb") -> Workload:
    return Workload("c1_gaussian_64_periodic", 64, 64, 2000, flux_a=(0.05, 0.05), A0=(0.01, 0.0, 0.01),
                    k0=1.0, k2=k2, phi0_kind="hill", extra={"sigma": 6.0})


def c2() -> Workload:
    return Workload("c2_aniso_1024_hbb", 1024, 1024, 20000, flux_a=(0.02, 0.0), A0=(0.02, 0.008, 0.01),
                    source=("sin", 1.0, 1, 1), bc_type=(DIRICHLET,) * 4, bc_value=(0.0,) * 4, k0=1.0, k2=1.0,
                    seed=2, phi0_kind="uniform")


def c3() -> Workload:
    return Workload("c3_nonlinear_4096_periodic", 4096, 4096, 5000, flux_b=(0.05, 0.05), A0=(0.01, 0.0, 0.005),
                    beta=1.0, k0=1.0, k2=1.0, seed=3, phi0_kind="gaussians", extra={"count": 16})


def c6(alpha: float = 1e-2, n: int = 50, t_end: float = 3.0, u=(0.1, 0.1), dt: Optional[float] = None) -> Workload:
    """Eqs. (73)-(76) on the unit square with N x N nodes, converted to lattice units."""
    dx = 1.0 / n
    dt = dx if dt is None else dt
    c = np.arange(n, dtype=np.float64) * dx + 0.5 * dx
    X, Y = np.meshgrid(c, c)
    sx, sy = np.sin(2 * np.pi * X), np.sin(2 * np.pi * Y)
    a_lat = alpha * dt / (dx * dx)
    field = np.zeros((n, n, 3))
    field[..., 0] = (2.0 - sx * sy) * a_lat
    field[..., 2] = a_lat
    # Eq. (75) without its time factor, times dt (the source per lattice step).
    s1 = (sx * sy + 4.0 * alpha * np.pi ** 2 * np.cos(4 * np.pi * X) * sy ** 2
          + 2.0 * np.pi * (u[0] * np.cos(2 * np.pi * X) * sy + u[1] * sx * np.cos(2 * np.pi * Y))) * dt
    lam = 1.0 - 12.0 * np.pi ** 2 * alpha
    steps = int(round(t_end / dt))
    return Workload(f"c6_var_tensor_{n}", n, n, steps, flux_a=(u[0] * dt / dx, u[1] * dt / dx),
                    A0=(0.0, 0.0, 0.0), source=("field", s1, lam * dt), A0_field=field, k0=1.0, k2=1.0,
                    phi0_kind="sin2", extra={"alpha": alpha, "dt": dt, "dx": dx, "lambda": lam})


def _bfe_wave(x, y, t, a, alpha, b, delta):
    """The travelling wave of Eqs. (68)-(69) (boundary and initial data of the bfe workload), with
    the speed a / (delta + 1) + 2 b alpha (delta + 1) / a that makes it solve Eq. (67) in 2-D."""
    k = -a * delta / (4.0 * alpha * (delta + 1.0))
    speed = (a * a + 2.0 * b * alpha * (delta + 1.0) ** 2) / (a * (delta + 1.0))
    return (0.5 + 0.5 * np.tanh(k * (x + y - speed * t))) ** (1.0 / delta)


def bfe(n: int = 40, alpha: float = 0.05, a: float = 2.0, b: float = 0.05, delta: float = 1.5, c: float = 5.0,
        t_end: float = 1.0) -> Workload:
    """The Burgers-Fisher problem on [-1, 2]^2 (Eqs. (67)-(69)), n nodes per unit length."""
    dx = 1.0 / n
    dt = dx / c
    m = 3 * n
    steps = int(round(t_end / dt))
    a_lat = alpha * dt / (dx * dx)

    # The 2m + 1 points along a side where links meet it: every half lattice spacing from one
    # corner to the other (the nodes' rows or columns and the points between them).
    along = -1.0 + np.arange(2 * m + 1, dtype=np.float64) * (0.5 * dx)

    def walls(k: int) -> np.ndarray:
        t = (k + 1) * dt
        lo, hi = np.full(2 * m + 1, -1.0), np.full(2 * m + 1, 2.0)
        return np.concatenate([_bfe_wave(lo, along, t, a, alpha, b, delta),
                               _bfe_wave(hi, along, t, a, alpha, b, delta),
                               _bfe_wave(along, lo, t, a, alpha, b, delta),
                               _bfe_wave(along, hi, t, a, alpha, b, delta)])

    bc0 = walls(-1)
    side = 2 * m + 1  # the initial per-side constants: each side's value at its first node
    return Workload(f"bfe_a{a:g}_alpha{alpha:g}_{m}", m, m, steps, A0=(a_lat, 0.0, a_lat),
                    bc_type=(DIRICHLET,) * 4, bc_value=(float(bc0[1]), float(bc0[side + 1]),
                                                        float(bc0[2 * side + 1]), float(bc0[3 * side + 1])),
                    k0=1.0, k2="hbb", phi0_kind="bfe",
                    flux_c=(a / ((delta + 1.0) * c), 0.0), flux_q=delta + 1.0, src_r=b * dt, src_p=delta,
                    walls=walls,
                    extra={"a": a, "alpha": alpha, "b": b, "delta": delta, "c": c, "dx": dx, "dt": dt,
                           "x0": -1.0})


def initial_field(w: Workload) -> np.ndarray:
    """phi0 on the cell-centred nodes (i + 1/2, j + 1/2), shape (ny, nx)."""
    x = np.arange(w.nx, dtype=np.float64) + 0.5
    y = np.arange(w.ny, dtype=np.float64) + 0.5
    X, Y = np.meshgrid(x, y)
    if w.phi0_kind == "uniform":
        return np.random.default_rng(w.seed).random((w.ny, w.nx))
    if w.phi0_kind == "hill":
        # Gaussian of unit peak at the box centre, summed over periodic images |m|,|n| <= 2.
        s = w.extra["sigma"]
        cx, cy = w.nx / 2.0, w.ny / 2.0
        out = np.zeros((w.ny, w.nx))
        for m in range(-2, 3):
            for n in range(-2, 3):
                out += np.exp(-((X - cx - m * w.nx) ** 2 + (Y - cy - n * w.ny) ** 2) / (2.0 * s * s))
        return out
    if w.phi0_kind == "gaussians":
        rng = np.random.default_rng(w.seed)
        k = w.extra["count"]
        amp = rng.uniform(0.0, 1.0, k)
        sig = rng.uniform(8.0, 64.0, k)
        # Centres scale with the box so scaled variants keep the same layout.
        cx = rng.uniform(0.0, 1.0, k) * w.nx
        cy = rng.uniform(0.0, 1.0, k) * w.ny
        sig = sig * max(min(w.nx, w.ny) / 4096.0, 0.125) if min(w.nx, w.ny) < 4096 else sig
        out = np.zeros((w.ny, w.nx))
        for a, s, x0, y0 in zip(amp, sig, cx, cy):
            dx = X - x0
            dx -= w.nx * np.round(dx / w.nx)
            dy = Y - y0
            dy -= w.ny * np.round(dy / w.ny)
            out += a * np.exp(-(dx * dx + dy * dy) / (2.0 * s * s))
        return out
    if w.phi0_kind == "bfe":
        e = w.extra
        c = e["x0"] + (np.arange(w.nx, dtype=np.float64) + 0.5) * e["dx"]
        Xp, Yp = np.meshgrid(c, c)
        return _bfe_wave(Xp, Yp, 0.0, e["a"], e["alpha"], e["b"], e["delta"])
    if w.phi0_kind == "sin2":
        # sin(2 pi x) sin(2 pi y) on the unit square (x = (i + 1/2) / nx).
        return np.sin(2 * np.pi * X / w.nx) * np.sin(2 * np.pi * Y / w.ny)
    raise ValueError(w.phi0_kind)


def c4(count: int = 256, seed: int = 4, steps: int = 2000, side_range=(32, 512)) -> list:
    """The batched workload: a list of independent square instances (see the module notes)."""
    rng = np.random.default_rng(seed)
    out = []
    lo, hi = np.log(side_range[0]), np.log(side_range[1])
    for k in range(count):
        n = int(round(np.exp(rng.uniform(lo, hi))))
        k11, k22 = rng.uniform(0.005, 0.05, 2)
        k12 = rng.uniform(-0.5, 0.5) * np.sqrt(k11 * k22)
        u = rng.uniform(-0.05, 0.05, 2)
        r0 = rng.uniform(0.0, 1e-4)
        if rng.random() < 0.5:
            bc_type, bc_value, src = (PERIODIC,) * 4, (0.0,) * 4, ("sin", r0, 2, 2)
        else:
            bc_type, bc_value, src = (DIRICHLET,) * 4, tuple(rng.uniform(0.0, 1.0, 4)), ("sin", r0, 1, 1)
        out.append(Workload(f"c4_{k:03d}_{n}", n, n, steps, flux_a=(float(u[0]), float(u[1])),
                            A0=(float(k11), float(k12), float(k22)), source=src, bc_type=bc_type,
                            bc_value=tuple(float(v) for v in bc_value), k0=1.0, k2=1.0,
                            seed=int(rng.integers(1 << 31)), phi0_kind="uniform"))
    return out


def c5(count: int, rate: float, seed: int = 5, side_range=(64, 2048), tol: float = 1e-8,
       max_steps: int = 50000) -> list:
    """Served requests: a list of (arrival time in seconds, Workload, tol, max_steps)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    base = c4(count=count, seed=seed + 1000, steps=max_steps, side_range=side_range)
    out = []
    for k, w in enumerate(base):
        t += rng.exponential(1.0 / rate)
        if rng.random() < 0.5:
            w.beta = 1.0
        w.name = f"c5_{k:04d}_{w.nx}"
        out.append((t, w, tol, max_steps))
    return out


@dataclass
class Workload3:
    """A D3Q19 problem in lattice units (faces x-, x+, y-, y+, z-, z+; A0 = (a11, a12, a13, a22, a23,
    a33)); phi0 and the source are (nz, ny, nx) arrays."""
    name: str
    nx: int
    ny: int
    nz: int
    steps: int
    flux_a: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    flux_b: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    A0: Tuple[float, ...] = (0.0,) * 6
    beta: float = 0.0
    source: Optional[np.ndarray] = None
    bc_type: Tuple[int, ...] = (PERIODIC,) * 6
    bc_value: Tuple[float, ...] = (0.0,) * 6
    k0: float = 1.0
    k2: object = 1.0
    phi0_array: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    def phi0(self) -> np.ndarray:
        return self.phi0_array


D3_A0 = np.array([[0.05, 0.01, 0.005], [0.01, 0.04, -0.008], [0.005, -0.008, 0.03]])


def _centres3(nx, ny, nz):
    return np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")


def d3_hill(n: int = 24, steps: Optional[int] = None) -> Workload3:
    """Periodic n^3 box, anisotropic A0, convection scaled with 16/n, the 3-D Gaussian of sigma n/6."""
    A = D3_A0
    u = np.array([0.02, -0.01, 0.015]) * 16 / n
    s0 = n / 6
    z, y, x = _centres3(n, n, n)
    phi0 = np.zeros((n, n, n))
    Si = np.eye(3) / s0 ** 2
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                d = np.stack([x - n / 2 - i * n, y - n / 2 - j * n, z - n / 2 - k * n])
                phi0 += np.exp(-0.5 * np.einsum("a...,ab,b...->...", d, Si, d))
    steps = int(round(40 * (n / 16) ** 2)) if steps is None else steps
    return Workload3(f"d3_hill_{n}", n, n, n, steps, flux_a=tuple(u), A0=(A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2],
                     A[2, 2]), phi0_array=phi0, extra={"sigma": s0, "u": u, "A": A})


def d3_nonlinear(nx: int = 256, ny: int = 256, nz: int = 256, steps: int = 200, seed: int = 7) -> Workload3:
    """Periodic box, Burgers-type flux plus linear convection, A(phi) = diag(0.01, 0.008, 0.006)(1 + phi^2),
    phi0 a seeded sum of 12 Gaussians (minimum image)."""
    rng = np.random.default_rng(seed)
    m = min(nx, ny, nz)
    amp = rng.uniform(0.0, 1.0, 12)
    sig = rng.uniform(0.06, 0.15, 12) * m
    cen = rng.uniform(0.0, 1.0, (12, 3)) * np.array([nx, ny, nz])
    phi0 = np.zeros((nz, ny, nx))
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    z = np.arange(nz) + 0.5
    for a, s, c in zip(amp, sig, cen):
        dx = x - c[0]
        dx -= nx * np.round(dx / nx)
        dy = y - c[1]
        dy -= ny * np.round(dy / ny)
        dz = z - c[2]
        dz -= nz * np.round(dz / nz)
        gx, gy, gz = np.exp(-dx * dx / (2 * s * s)), np.exp(-dy * dy / (2 * s * s)), np.exp(-dz * dz / (2 * s * s))
        phi0 += a * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return Workload3(f"d3_nonlinear_{nx}x{ny}x{nz}", nx, ny, nz, steps, flux_a=(0.01, 0.0, -0.01),
                     flux_b=(0.025, 0.025, 0.025), A0=(0.01, 0.0, 0.0, 0.008, 0.0, 0.006), beta=1.0, phi0_array=phi0)


def d3_walls(nx: int = 37, ny: int = 29, nz: int = 23, steps: int = 120, seed: int = 8) -> Workload3:
    """Six Dirichlet faces, full anisotropic A0 with beta = 0.5, a sine source, random phi0."""
    z, y, x = _centres3(nx, ny, nz)
    S = 1e-3 * np.sin(np.pi * x / nx) * np.sin(np.pi * y / ny) * np.sin(np.pi * z / nz)
    phi0 = np.random.default_rng(seed).random((nz, ny, nx))
    A = D3_A0
    return Workload3(f"d3_walls_{nx}x{ny}x{nz}", nx, ny, nz, steps, flux_a=(0.02, 0.01, -0.015),
                     flux_b=(0.01, 0.0, 0.0), A0=(A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]), beta=0.5,
                     source=S, bc_type=(DIRICHLET,) * 6, bc_value=(0.2, 0.5, 0.3, 0.6, 0.4, 0.1),
                     k2=(0.9, 1.1, 1.0, 1.2, 1.3, 0.95, 1.05, 0.85, 1.15), phi0_array=phi0)
