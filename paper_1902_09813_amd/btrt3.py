"""ctypes binding of include/btrt3.h: the D3Q19 solver of libbtrt.so (argument marshalling only;
every step of the method runs in the library's kernels, and the binding raises if the library
is not built)."""
from __future__ import annotations

import ctypes

import numpy as np

from paper_1902_09813_amd.btrt import (BtrtError, F32, F64, K2_HBB, K2_VALUE, SRC_FIELD, SRC_NONE, _check, _dptr,
                                        lib as _lib2)

# Every function include/btrt3.h declares.
EXPORTS = ("btrt3_validate", "btrt3_create", "btrt3_step", "btrt3_set_launch", "btrt3_get_launch", "btrt3_field",
           "btrt3_populations", "btrt3_residual", "btrt3_error", "btrt3_solve", "btrt3_sync", "btrt3_get_info",
           "btrt3_destroy")

__all__ = ["Problem3", "Solver3", "problem_from_workload3", "BtrtError", "F64", "F32", "EXPORTS"]


class Grid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("device", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class Flux3(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double * 3), ("b", ctypes.c_double * 3)]


class Diff3(ctypes.Structure):
    _fields_ = [("a0", ctypes.c_double * 6), ("beta", ctypes.c_double)]


class Source3(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("field", ctypes.POINTER(ctypes.c_double))]


class BC3(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32 * 6), ("value", ctypes.c_double * 6)]


class Relax3(ctypes.Structure):
    _fields_ = [("k0", ctypes.c_double), ("k2_rule", ctypes.c_int32), ("k2", ctypes.c_double * 9),
                ("check_interval", ctypes.c_int32)]


class Launch3(ctypes.Structure):
    _fields_ = [("steps_per_launch", ctypes.c_int32), ("z_chunk", ctypes.c_int32), ("tile", ctypes.c_int32)]

    def as_tuple(self):
        return (self.steps_per_launch, self.z_chunk, self.tile)


class Info3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("pitch", ctypes.c_int32), ("k1_per_node", ctypes.c_int32),
                ("K1", ctypes.c_double * 9), ("K2", ctypes.c_double * 9), ("k0", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t), ("bytes_per_node_launch", ctypes.c_double),
                ("step", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        L = _lib2()
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        hp = ctypes.c_void_p
        sig = {
            "btrt3_validate": ([P(Grid3), P(Flux3), P(Diff3), P(Source3), P(BC3), P(Relax3), P(Info3)], ctypes.c_int),
            "btrt3_create": ([P(Grid3), P(Flux3), P(Diff3), P(Source3), P(BC3), P(Relax3), dp, P(hp)], ctypes.c_int),
            "btrt3_step": ([hp, ctypes.c_int64], ctypes.c_int),
            "btrt3_set_launch": ([hp, P(Launch3)], ctypes.c_int),
            "btrt3_get_launch": ([hp, P(Launch3)], ctypes.c_int),
            "btrt3_field": ([hp, dp], ctypes.c_int),
            "btrt3_populations": ([hp, dp], ctypes.c_int),
            "btrt3_residual": ([hp, dp], ctypes.c_int),
            "btrt3_error": ([hp, dp, dp], ctypes.c_int),
            "btrt3_solve": ([hp, ctypes.c_double, ctypes.c_int64, P(ctypes.c_int64), dp], ctypes.c_int),
            "btrt3_sync": ([hp], ctypes.c_int),
            "btrt3_get_info": ([hp, P(Info3)], ctypes.c_int),
            "btrt3_destroy": ([hp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class Problem3:
    """The arguments of btrt3_create: flux_a, flux_b (B = a phi + b phi^2 / 2), A0 =
    (a11, a12, a13, a22, a23, a33) and beta (A = A0 (1 + beta phi^2)), source None or an
    (nz, ny, nx) array, faces x-, x+, y-, y+, z-, z+, k0 and k2 ("hbb", a scalar or nine entries)."""

    def __init__(self, nx: int, ny: int, nz: int, *, precision: int = F64, flux_a=(0.0, 0.0, 0.0),
                 flux_b=(0.0, 0.0, 0.0), A0=(0.0,) * 6, beta: float = 0.0, source=None, bc_type=(0,) * 6,
                 bc_value=(0.0,) * 6, k0: float = 1.0, k2=1.0, check_interval: int = 1000, device: int = 0):
        self.grid = Grid3(int(nx), int(ny), int(nz), int(precision), int(device), None)
        self.flux = Flux3((ctypes.c_double * 3)(*flux_a), (ctypes.c_double * 3)(*flux_b))
        self.diff = Diff3((ctypes.c_double * 6)(*A0), float(beta))
        self._field = None
        if source is None:
            self.source = Source3(SRC_NONE, None)
        else:
            self._field = np.ascontiguousarray(source, dtype=np.float64).reshape(nz, ny, nx)
            self.source = Source3(SRC_FIELD, _dptr(self._field))
        self.bc = BC3((ctypes.c_int32 * 6)(*bc_type), (ctypes.c_double * 6)(*bc_value))
        if isinstance(k2, str):
            assert k2 == "hbb"
            self.relax = Relax3(float(k0), K2_HBB, (ctypes.c_double * 9)(*([0.0] * 9)), int(check_interval))
        else:
            vals = [float(k2)] * 9 if np.isscalar(k2) else [float(v) for v in k2]
            self.relax = Relax3(float(k0), K2_VALUE, (ctypes.c_double * 9)(*vals), int(check_interval))

    @property
    def shape(self):
        return (self.grid.nz, self.grid.ny, self.grid.nx)

    def args(self):
        b = ctypes.byref
        return (b(self.grid), b(self.flux), b(self.diff), b(self.source), b(self.bc), b(self.relax))

    def validate(self) -> Info3:
        info = Info3()
        _check(lib().btrt3_validate(*self.args(), ctypes.byref(info)), "btrt3_validate")
        return info


class Solver3:
    """One btrt3 handle."""

    def __init__(self, problem: Problem3, phi0: np.ndarray):
        self.problem = problem
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(problem.shape)
        h = ctypes.c_void_p()
        _check(lib().btrt3_create(*problem.args(), _dptr(phi0), ctypes.byref(h)), "btrt3_create")
        self.h = h

    def step(self, n: int) -> "Solver3":
        _check(lib().btrt3_step(self.h, int(n)), "btrt3_step")
        return self

    def set_launch(self, steps_per_launch: int, z_chunk: int = 0, tile: int = 0) -> "Solver3":
        cfg = Launch3(int(steps_per_launch), int(z_chunk), int(tile))
        _check(lib().btrt3_set_launch(self.h, ctypes.byref(cfg)), "btrt3_set_launch")
        return self

    def launch(self):
        """(steps_per_launch, z_chunk, tile) in force, automatic fields resolved."""
        cfg = Launch3()
        _check(lib().btrt3_get_launch(self.h, ctypes.byref(cfg)), "btrt3_get_launch")
        return cfg.as_tuple()

    def field(self) -> np.ndarray:
        out = np.empty(self.problem.shape)
        _check(lib().btrt3_field(self.h, _dptr(out)), "btrt3_field")
        return out

    def populations(self) -> np.ndarray:
        out = np.empty((19,) + self.problem.shape)
        _check(lib().btrt3_populations(self.h, _dptr(out)), "btrt3_populations")
        return out

    def residual(self) -> float:
        v = ctypes.c_double()
        _check(lib().btrt3_residual(self.h, ctypes.byref(v)), "btrt3_residual")
        return float(v.value)

    def error(self, ref: np.ndarray):
        ref = np.ascontiguousarray(ref, dtype=np.float64).reshape(self.problem.shape)
        out = np.empty(3)
        _check(lib().btrt3_error(self.h, _dptr(ref), _dptr(out)), "btrt3_error")
        return tuple(out)

    def solve(self, tol: float, max_steps: int):
        n = ctypes.c_int64()
        r = ctypes.c_double()
        _check(lib().btrt3_solve(self.h, float(tol), int(max_steps), ctypes.byref(n), ctypes.byref(r)), "btrt3_solve")
        return int(n.value), float(r.value)

    def sync(self) -> None:
        _check(lib().btrt3_sync(self.h), "btrt3_sync")

    def info(self) -> Info3:
        info = Info3()
        _check(lib().btrt3_get_info(self.h, ctypes.byref(info)), "btrt3_get_info")
        return info

    def close(self) -> None:
        if getattr(self, "h", None):
            _check(lib().btrt3_destroy(self.h), "btrt3_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def problem_from_workload3(w, precision: int = F64, device: int = 0, check_interval: int = 1000) -> Problem3:
    """btrt3_create arguments for a workloads.Workload3."""
    return Problem3(w.nx, w.ny, w.nz, precision=precision, flux_a=w.flux_a, flux_b=w.flux_b, A0=w.A0, beta=w.beta,
                    source=w.source, bc_type=w.bc_type, bc_value=w.bc_value, k0=w.k0, k2=w.k2,
                    check_interval=check_interval, device=device)
