"""Python side of the FP64 CPU oracle of the B-TriRT D2Q9 scheme (arXiv:1902.09813).

TEST INFRASTRUCTURE: only the tests, the package's smoke check and the
benchmark's CPU-baseline leg import this module. It loads the plain-C oracle
(btrt_oracle.c) and adds the paper's scalar formulas and closed-form
solutions used as pins:

* ``k1_isotropic``         Eq. (30) for A = alpha I.
* ``k2_hbb``               Eq. (62), the k2 that removes the bounce-back slip.
* ``hbb_slip``             Eq. (61), the numerical slip of half-way bounce-back.
* ``gre``                  Eq. (63), global relative error.
* ``residual``             Eq. (64), relative L1 change used as the steady criterion.
* ``gaussian_hill``        Eq. (71), the anisotropic Gaussian hill (with periodic images).
* ``source_sin``           the separable sinusoidal source of the benchmark problems.
* ``burgers_fisher``       Eqs. (68)-(69), the travelling wave of the Burgers-Fisher equation.
* ``WallLinks``            per-link Dirichlet values at the points where links cross the walls.

Nothing here imports the product package.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_btrt.so")

PERIODIC = 0
DIRICHLET = 1


class _CProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("flux_a", ctypes.c_double * 2),
        ("flux_b", ctypes.c_double * 2),
        ("A0", ctypes.c_double * 3),
        ("beta", ctypes.c_double),
        ("k0", ctypes.c_double),
        ("K2", ctypes.c_double * 4),
        ("bc_type", ctypes.c_int * 4),
        ("bc_value", ctypes.c_double * 4),
        ("A0_field", ctypes.POINTER(ctypes.c_double)),
        ("flux_c", ctypes.c_double * 2),
        ("flux_q", ctypes.c_double),
        ("src_r", ctypes.c_double),
        ("src_p", ctypes.c_double),
        ("d_kind", ctypes.c_int),
        ("d_g", ctypes.c_double),
        ("d_e", ctypes.c_double),
        ("d_s", ctypes.c_double),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load the compiled oracle (building it first if nothing is built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b  # noqa: WPS433
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_CProblem)
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp, dp]
        L.orc_equilibrium.restype = None
        L.orc_collide_node.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_collide_node.restype = None
        L.orc_init.argtypes = [pp, dp, dp]
        L.orc_init.restype = None
        L.orc_phi.argtypes = [pp, dp, dp]
        L.orc_phi.restype = None
        L.orc_run.argtypes = [pp, dp, dp, dp, dp, dp, dp, ctypes.c_long, ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_threads.argtypes = [ctypes.c_int]
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Problem:
    """One B-TriRT problem in lattice units (Eq. (1) with D = phi I).

    flux:   B(phi) = a phi + b phi^2 / 2 + c |phi|^q per component.
    A0, beta: A(phi) = A0 (1 + beta phi^2), A0 = (a11, a12, a22) symmetric.
    k0, K2: relaxation of the S0 block and the 2x2 K2 block of Eq. (6) (row major).
    bc_type/bc_value: sides x-, x+, y-, y+.
    src_r, src_p: phi-dependent source r phi (1 - |phi|^p), added to any given S.
    dterm: None for D = phi I, or (g, e, s) for D = (g phi + e |phi|^s) I (Eq. (1), Eq. (7)).
    """

    nx: int
    ny: int
    flux_a: Sequence[float] = (0.0, 0.0)
    flux_b: Sequence[float] = (0.0, 0.0)
    A0: Sequence[float] = (0.0, 0.0, 0.0)
    beta: float = 0.0
    k0: float = 1.0
    K2: Sequence[float] = (1.0, 1.0, 1.0, 1.0)
    bc_type: Sequence[int] = (PERIODIC,) * 4
    bc_value: Sequence[float] = (0.0,) * 4
    A0_field: Optional[np.ndarray] = None  # (ny, nx, 3): space-dependent A0(x) (Eq. (74))
    flux_c: Sequence[float] = (0.0, 0.0)
    flux_q: float = 1.0
    src_r: float = 0.0
    src_p: float = 1.0
    dterm: Optional[Sequence[float]] = None

    def c(self) -> _CProblem:
        p = _CProblem()
        p.nx, p.ny = int(self.nx), int(self.ny)
        p.flux_a[:] = [float(v) for v in self.flux_a]
        p.flux_b[:] = [float(v) for v in self.flux_b]
        p.A0[:] = [float(v) for v in self.A0]
        p.beta = float(self.beta)
        p.k0 = float(self.k0)
        K2 = list(self.K2)
        if len(K2) == 1:
            K2 = K2 * 4
        p.K2[:] = [float(v) for v in K2]
        p.bc_type[:] = [int(v) for v in self.bc_type]
        p.bc_value[:] = [float(v) for v in self.bc_value]
        p.flux_c[:] = [float(v) for v in self.flux_c]
        p.flux_q = float(self.flux_q)
        p.src_r = float(self.src_r)
        p.src_p = float(self.src_p)
        if self.dterm is not None:
            p.d_kind = 1
            p.d_g, p.d_e, p.d_s = (float(v) for v in self.dterm)
        if self.A0_field is not None:
            field = np.ascontiguousarray(self.A0_field, dtype=np.float64)
            assert field.shape == (self.ny, self.nx, 3)
            p._field = field  # keeps the array alive as long as the structure
            p.A0_field = field.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return p


class Oracle:
    """State of one oracle run: post-streaming populations f(t) and phi(t-1)."""

    def __init__(self, problem: Problem, phi0: np.ndarray, source: Optional[np.ndarray] = None,
                 nthreads: int = 0):
        self.problem = problem
        self._cp = problem.c()
        ny, nx = problem.ny, problem.nx
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(ny, nx)
        self.f = np.empty((9, ny, nx), dtype=np.float64)
        self.work = np.empty_like(self.f)
        # Reading of Eq. (11) at the first step: phi(-1) := phi(0), so G vanishes.
        self.phi_prev = phi0.copy()
        self.source = None if source is None else np.ascontiguousarray(source, dtype=np.float64).reshape(ny, nx)
        self.nthreads = nthreads
        self.t = 0
        lib().orc_init(ctypes.byref(self._cp), _ptr(phi0), _ptr(self.f))

    def step(self, n: int = 1, S: Optional[np.ndarray] = None, S_prev: Optional[np.ndarray] = None,
             wall: Optional[np.ndarray] = None) -> "Oracle":
        """Advance n steps. S/S_prev override the stored time-independent source;
        ``wall`` (9, ny, nx) gives per-link Dirichlet values (see orc_run)."""
        if S is None:
            S = self.source
        if S is not None:
            S = np.ascontiguousarray(S, dtype=np.float64)
        if S_prev is not None:
            S_prev = np.ascontiguousarray(S_prev, dtype=np.float64)
        if wall is not None:
            wall = np.ascontiguousarray(wall, dtype=np.float64)
            assert wall.shape == self.f.shape
        rc = lib().orc_run(ctypes.byref(self._cp), _ptr(self.f), _ptr(self.work), _ptr(self.phi_prev),
                           _ptr(S), _ptr(S_prev), _ptr(wall), int(n), int(self.nthreads))
        if rc != 0:
            raise ValueError("oracle rejected the problem")
        self.t += n
        return self

    def phi(self) -> np.ndarray:
        out = np.empty((self.problem.ny, self.problem.nx), dtype=np.float64)
        lib().orc_phi(ctypes.byref(self._cp), _ptr(self.f), _ptr(out))
        return out


def collide_node(problem: Problem, f: np.ndarray, phi_prev: float, S: float = 0.0,
                 S_prev: Optional[float] = None) -> np.ndarray:
    """One node of Eq. (6) (f -> f+), for unit tests."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(9, dtype=np.float64)
    cp = problem.c()
    lib().orc_collide_node(ctypes.byref(cp), _ptr(f), float(phi_prev), float(S),
                           float(S if S_prev is None else S_prev), _ptr(out))
    return out


def equilibrium(phi: float, B: Sequence[float], D: Sequence[float]) -> np.ndarray:
    """Eq. (7) for one node."""
    Bv = np.ascontiguousarray(B, dtype=np.float64)
    Dv = np.ascontiguousarray(D, dtype=np.float64)
    out = np.empty(9, dtype=np.float64)
    lib().orc_equilibrium(float(phi), _ptr(Bv), _ptr(Dv), _ptr(out))
    return out


def threads(nthreads: int = 0) -> int:
    return int(lib().orc_threads(int(nthreads)))


# ----------------------------------------------------------------------------------------
# Scalar formulas and closed forms of the paper.
# ----------------------------------------------------------------------------------------

def k1_isotropic(alpha: float) -> float:
    """Eq. (30) for A = alpha I in lattice units: k1 = 1 / (alpha / c_s^2 + 1/2)."""
    return 1.0 / (3.0 * alpha + 0.5)


def k2_hbb(k1: float) -> float:
    """Eq. (62): k2 = 8 (k1 - 2) / (3 (k1 - 4))."""
    return 8.0 * (k1 - 2.0) / (3.0 * (k1 - 4.0))


def hbb_slip(k1: float, k2: float, dphi: float, N: int) -> float:
    """Eq. (61): slip of the half-way bounce-back steady solution."""
    return (3.0 * k1 * k2 - 8.0 * k1 - 12.0 * k2 + 16.0) / (12.0 * k1 * k2) * dphi / N ** 2


def gre(phi: np.ndarray, ref: np.ndarray) -> float:
    """Eq. (63): sum |phi - phi*| / sum |phi*|."""
    return float(np.sum(np.abs(phi - ref)) / np.sum(np.abs(ref)))


def residual(phi_new: np.ndarray, phi_old: np.ndarray) -> float:
    """Eq. (64): sum |phi(t+T) - phi(t)| / sum |phi(t+T)|."""
    return float(np.sum(np.abs(phi_new - phi_old)) / np.sum(np.abs(phi_new)))


def cell_centres(nx: int, ny: int):
    """Cell-centred node coordinates (x_i = i + 1/2), as for y_n = (n - 1/2)/N below Eq. (49)."""
    x = np.arange(nx, dtype=np.float64) + 0.5
    y = np.arange(ny, dtype=np.float64) + 0.5
    return np.meshgrid(x, y)


def source_sin(nx: int, ny: int, amp: float, kx: int, ky: int) -> np.ndarray:
    """amp sin(kx pi x / nx) sin(ky pi y / ny) at cell centres."""
    X, Y = cell_centres(nx, ny)
    return amp * np.sin(kx * np.pi * X / nx) * np.sin(ky * np.pi * Y / ny)


def gaussian_hill(nx: int, ny: int, t: float, x0: Sequence[float], sigma0: float,
                  u: Sequence[float], A: np.ndarray, amp: float = 1.0, images: int = 2) -> np.ndarray:
    """Eq. (71) scaled to peak value ``amp`` at t = 0, on a periodic nx x ny box.

    sigma_t = sigma0^2 I + 2 A t; phi = amp sigma0^2 / sqrt(det sigma_t)
    exp(-(x - x0 - u t)^T sigma_t^{-1} (x - x0 - u t) / 2), summed over the periodic
    images |m|, |n| <= images.
    """
    A = np.asarray(A, dtype=np.float64).reshape(2, 2)
    st = sigma0 ** 2 * np.eye(2) + 2.0 * A * t
    si = np.linalg.inv(st)
    pref = amp * sigma0 ** 2 / np.sqrt(abs(np.linalg.det(st)))
    X, Y = cell_centres(nx, ny)
    cx = x0[0] + u[0] * t
    cy = x0[1] + u[1] * t
    out = np.zeros((ny, nx))
    for m in range(-images, images + 1):
        for n in range(-images, images + 1):
            dx = X - cx - m * nx
            dy = Y - cy - n * ny
            q = si[0, 0] * dx * dx + (si[0, 1] + si[1, 0]) * dx * dy + si[1, 1] * dy * dy
            out += np.exp(-0.5 * q)
    return pref * out


def burgers_fisher(X, Y, t: float, a: float, alpha: float, b: float, delta: float) -> np.ndarray:
    """Eqs. (68)-(69): {1/2 + tanh[A (x + y - omega t)] / 2}^(1/delta) with
    A = -a delta / (4 alpha (delta + 1)) and omega = a / (delta + 1) + 2 b alpha (delta + 1) / a.

    The speed printed with Eq. (69) has (delta + 1) where this one has (delta + 1)^2 in the
    b alpha term; substituting the wave into Eq. (67) (where the diffusion acts along x + y with
    coefficient 2 alpha) leaves a residual unless the square is there, so the square is read
    as intended."""
    A = -a * delta / (4.0 * alpha * (delta + 1.0))
    omega = a / (delta + 1.0) + 2.0 * b * alpha * (delta + 1.0) / a
    return (0.5 + 0.5 * np.tanh(A * (np.asarray(X) + np.asarray(Y) - omega * t))) ** (1.0 / delta)


class WallLinks:
    """Per-link Dirichlet values (9, ny, nx) for orc_run from values sampled along the sides.

    Half-way bounce-back (Eqs. (54)-(56)) puts the wall half a lattice spacing beyond the last
    node, so the link from node x along c_i meets it at x + c_i/2. With the node of column i at
    i + 1/2 (and of row j at j + 1/2), the points where links meet a side lie at half-integer
    and integer positions along it: a side of n nodes carries 2n + 1 samples, sample s at
    position s/2 measured from the side's lower corner (odd s: level with a node; even s: between
    two nodes; s = 0 and s = 2n: the corners). The vector v holds, in order, x- (2 ny + 1 samples
    along y), x+ (2 ny + 1), y- (2 nx + 1 samples along x), y+ (2 nx + 1).

    The link from node (i, j) along c = (cx, cy) that leaves through x- or x+ takes that side's
    sample 2 j + 1 + cy; through y- or y+, the sample 2 i + 1 + cx. A diagonal link from a corner
    node that leaves through both (it meets the corner point) takes the mean of the two sides'
    corner samples, which is the corner value itself when the two sides agree there and the mean
    of the two sides for unequal constant sides.
    """

    CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
    CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)

    def __init__(self, nx: int, ny: int, bc_type: Sequence[int]):
        self.nx, self.ny = nx, ny
        perx, pery = bc_type[0] == PERIODIC, bc_type[2] == PERIODIC
        base = {"x-": 0, "x+": 2 * ny + 1, "y-": 2 * (2 * ny + 1), "y+": 2 * (2 * ny + 1) + 2 * nx + 1}
        links, ia, ib = [], [], []
        edge = sorted({(i, j) for j in range(ny) for i in (0, nx - 1)}
                      | {(i, j) for i in range(nx) for j in (0, ny - 1)}, key=lambda q: (q[1], q[0]))
        for k in range(1, 9):
            cx, cy = self.CX[k], self.CY[k]
            for i, j in edge:
                outx = not perx and not (0 <= i + cx < nx)
                outy = not pery and not (0 <= j + cy < ny)
                if not (outx or outy):
                    continue
                sx = base["x-" if cx < 0 else "x+"] + 2 * j + 1 + cy if outx else -1
                sy = base["y-" if cy < 0 else "y+"] + 2 * i + 1 + cx if outy else -1
                links.append((k * ny + j) * nx + i)
                ia.append(sx if outx else sy)
                ib.append(sy if outy else sx)
        self.size = 4 * (nx + ny) + 4
        self.links = np.asarray(links, dtype=np.int64)
        self.ia = np.asarray(ia, dtype=np.int64)
        self.ib = np.asarray(ib, dtype=np.int64)
        self.out = np.zeros((9, ny, nx))

    def __call__(self, v: np.ndarray) -> np.ndarray:
        v = np.asarray(v, dtype=np.float64)
        assert v.shape == (self.size,)
        flat = self.out.reshape(-1)
        flat[self.links] = 0.5 * (v[self.ia] + v[self.ib])
        return self.out

    def positions(self):
        """Lattice coordinates (x, y) of the 4 (nx + ny) + 4 samples of v, in v's order (walls at
        0 and nx, 0 and ny; nodes at i + 1/2)."""
        nx, ny = self.nx, self.ny
        sy = np.arange(2 * ny + 1) / 2.0
        sx = np.arange(2 * nx + 1) / 2.0
        xs = np.concatenate([np.zeros_like(sy), np.full_like(sy, nx), sx, sx])
        ys = np.concatenate([sy, sy, np.zeros_like(sx), np.full_like(sx, ny)])
        return xs, ys
