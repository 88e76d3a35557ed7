"""Python side of the FP64 CPU oracle of the three-dimensional B-TriRT scheme on D3Q19
(arXiv:1902.09813, Eq. (6) with the D3Q19 lattice of Eq. (86)).

TEST INFRASTRUCTURE: only the tests, the package's smoke check and the benchmark's
CPU-baseline leg import this module. It loads the plain-C oracle (btrt3_oracle.c, built
into the same library as the D2Q9 oracle) and adds the closed form used as a pin:

* ``gaussian_hill3``   the anisotropic Gaussian hill in 3-D (Eq. (71) with a 3x3 tensor),
                       summed over periodic images.

Nothing here imports the product package.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from oracle.oracle import lib as _lib2, _ptr

# D3Q19 velocities in the column order of Eq. (86), and the weights.
CX = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])
CY = np.array([0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1])
CZ = np.array([0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1])
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


class _CProblem3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("flux_a", ctypes.c_double * 3), ("flux_b", ctypes.c_double * 3),
        ("A0", ctypes.c_double * 6), ("beta", ctypes.c_double),
        ("k0", ctypes.c_double), ("K2", ctypes.c_double * 9),
        ("bc_type", ctypes.c_int * 6), ("bc_value", ctypes.c_double * 6),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        L = _lib2()
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_CProblem3)
        L.orc3_equilibrium.argtypes = [ctypes.c_double, dp, dp, dp]
        L.orc3_equilibrium.restype = None
        L.orc3_collide_node.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc3_collide_node.restype = None
        L.orc3_init.argtypes = [pp, dp, dp]
        L.orc3_init.restype = None
        L.orc3_phi.argtypes = [pp, dp, dp]
        L.orc3_phi.restype = None
        L.orc3_run.argtypes = [pp, dp, dp, dp, dp, dp, ctypes.c_long, ctypes.c_int]
        L.orc3_run.restype = ctypes.c_int
        _lib = L
    return _lib


@dataclass
class Problem3:
    """One D3Q19 problem in lattice units (Eq. (1) with D = phi I).

    flux: B(phi) = a phi + b phi^2 / 2; A0 = (a11, a12, a13, a22, a23, a33), beta: A = A0 (1 + beta
    phi^2); k0 and the 3x3 K2 (row major, or one value for all entries); faces x-, x+, y-, y+, z-, z+.
    """

    nx: int
    ny: int
    nz: int
    flux_a: Sequence[float] = (0.0, 0.0, 0.0)
    flux_b: Sequence[float] = (0.0, 0.0, 0.0)
    A0: Sequence[float] = (0.0,) * 6
    beta: float = 0.0
    k0: float = 1.0
    K2: Sequence[float] = (1.0,) * 9
    bc_type: Sequence[int] = (0,) * 6
    bc_value: Sequence[float] = (0.0,) * 6

    def c(self) -> _CProblem3:
        p = _CProblem3()
        p.nx, p.ny, p.nz = int(self.nx), int(self.ny), int(self.nz)
        p.flux_a[:] = [float(v) for v in self.flux_a]
        p.flux_b[:] = [float(v) for v in self.flux_b]
        p.A0[:] = [float(v) for v in self.A0]
        p.beta = float(self.beta)
        p.k0 = float(self.k0)
        K2 = list(self.K2)
        p.K2[:] = [float(v) for v in (K2 * 9 if len(K2) == 1 else K2)]
        p.bc_type[:] = [int(v) for v in self.bc_type]
        p.bc_value[:] = [float(v) for v in self.bc_value]
        return p


class Oracle3:
    """Post-streaming populations f(t) (19, nz, ny, nx) and phi(t-1)."""

    def __init__(self, problem: Problem3, phi0: np.ndarray, source: Optional[np.ndarray] = None, nthreads: int = 0):
        self.problem = problem
        self._cp = problem.c()
        shape = (problem.nz, problem.ny, problem.nx)
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(shape)
        self.f = np.empty((19,) + shape)
        self.work = np.empty_like(self.f)
        self.phi_prev = phi0.copy()
        self.source = None if source is None else np.ascontiguousarray(source, dtype=np.float64).reshape(shape)
        self.nthreads = nthreads
        self.t = 0
        lib().orc3_init(ctypes.byref(self._cp), _ptr(phi0), _ptr(self.f))

    def step(self, n: int = 1) -> "Oracle3":
        rc = lib().orc3_run(ctypes.byref(self._cp), _ptr(self.f), _ptr(self.work), _ptr(self.phi_prev),
                            _ptr(self.source), None, int(n), int(self.nthreads))
        if rc != 0:
            raise ValueError("oracle rejected the problem")
        self.t += n
        return self

    def phi(self) -> np.ndarray:
        out = np.empty((self.problem.nz, self.problem.ny, self.problem.nx))
        lib().orc3_phi(ctypes.byref(self._cp), _ptr(self.f), _ptr(out))
        return out


def collide_node(problem: Problem3, f: np.ndarray, phi_prev: float, S: float = 0.0,
                 S_prev: Optional[float] = None) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(19)
    cp = problem.c()
    lib().orc3_collide_node(ctypes.byref(cp), _ptr(f), float(phi_prev), float(S),
                            float(S if S_prev is None else S_prev), _ptr(out))
    return out


def equilibrium(phi: float, B: Sequence[float], D: Sequence[float]) -> np.ndarray:
    Bv = np.ascontiguousarray(B, dtype=np.float64)
    Dv = np.ascontiguousarray(D, dtype=np.float64)
    out = np.empty(19)
    lib().orc3_equilibrium(float(phi), _ptr(Bv), _ptr(Dv), _ptr(out))
    return out


def gaussian_hill3(n: Sequence[int], t: float, x0: Sequence[float], sigma0: float, u: Sequence[float],
                   A: np.ndarray, images: int = 1) -> np.ndarray:
    """The 3-D anisotropic Gaussian of unit peak at t = 0 on a periodic box of n = (nx, ny, nz)
    cell-centred nodes: sigma0^3 / sqrt(det S_t) exp(-(x - x0 - u t)^T S_t^-1 (x - x0 - u t) / 2),
    S_t = sigma0^2 I + 2 A t, summed over the periodic images within `images` boxes."""
    A = np.asarray(A, dtype=np.float64).reshape(3, 3)
    St = sigma0 ** 2 * np.eye(3) + 2.0 * A * t
    Si = np.linalg.inv(St)
    pref = sigma0 ** 3 / np.sqrt(np.linalg.det(St))
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    c = [x0[a] + u[a] * t for a in range(3)]
    out = np.zeros((nz, ny, nx))
    r = range(-images, images + 1)
    for i in r:
        for j in r:
            for k in r:
                d = np.stack([x - c[0] - i * nx, y - c[1] - j * ny, z - c[2] - k * nz])
                q = np.einsum("a...,ab,b...->...", d, Si, d)
                out += np.exp(-0.5 * q)
    return pref * out
