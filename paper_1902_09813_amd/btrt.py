"""ctypes binding of libbtrt (include/btrt.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels. PyTorch, when used, only
provides device memory (a workspace tensor) and the HIP stream the library enqueues on.
The binding fails loudly when the library is not built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbtrt.so")

# Constants of include/btrt.h.
OK, E_INVAL, E_NOMEM, E_DEVICE, E_UNSTABLE, E_STATE = 0, 1, 2, 3, 4, 5
F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
PERIODIC, DIRICHLET = 0, 1
SRC_NONE, SRC_FIELD, SRC_SIN = 0, 1, 2
D_PHI_I, D_POLY = 0, 1
K2_VALUE, K2_HBB = 0, 1

# Every function include/btrt.h declares.
EXPORTS = ("btrt_validate", "btrt_workspace_size", "btrt_create", "btrt_step", "btrt_set_walls", "btrt_set_launch",
           "btrt_get_launch",
           "btrt_set_fusion", "btrt_tune", "btrt_field",
           "btrt_populations", "btrt_residual", "btrt_error", "btrt_solve", "btrt_sync",
           "btrt_get_info", "btrt_destroy", "btrt_strerror", "btrt_last_error",
           "btrt_checkpoint_size", "btrt_checkpoint", "btrt_restore",
           "btrt_batch_create", "btrt_batch_step", "btrt_batch_field", "btrt_batch_residual",
           "btrt_batch_set_config", "btrt_batch_get_config", "btrt_batch_tune", "btrt_batch_steps",
           "btrt_batch_sync", "btrt_batch_destroy",
           "btrt_server_create", "btrt_server_submit", "btrt_server_pump", "btrt_server_info",
           "btrt_server_result", "btrt_server_stats", "btrt_server_clock", "btrt_server_destroy",
           "btrt_solve_static")


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class Flux(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double * 2), ("b", ctypes.c_double * 2), ("c", ctypes.c_double * 2),
                ("q", ctypes.c_double)]


class Diff(ctypes.Structure):
    _fields_ = [("k11", ctypes.c_double), ("k12", ctypes.c_double), ("k22", ctypes.c_double),
                ("beta", ctypes.c_double), ("field", ctypes.POINTER(ctypes.c_double))]


class DTerm(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("g", ctypes.c_double), ("e", ctypes.c_double), ("s", ctypes.c_double)]


class Source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("amp", ctypes.c_double), ("kx", ctypes.c_int32),
                ("ky", ctypes.c_int32), ("field", ctypes.POINTER(ctypes.c_double)), ("growth", ctypes.c_double),
                ("r", ctypes.c_double), ("p", ctypes.c_double)]


class BC(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32 * 4), ("value", ctypes.c_double * 4)]


class Relax(ctypes.Structure):
    _fields_ = [("k0", ctypes.c_double), ("k2_rule", ctypes.c_int32), ("k2", ctypes.c_double * 4),
                ("check_interval", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("k1_per_node", ctypes.c_int32), ("K1", ctypes.c_double * 4),
                ("K2", ctypes.c_double * 4), ("k0", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t),
                ("bytes_per_node_launch", ctypes.c_double), ("step", ctypes.c_int64)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("grid", Grid), ("B", Flux), ("K", Diff), ("D", DTerm), ("R", Source), ("bc", BC),
                ("relax", Relax), ("phi0", ctypes.POINTER(ctypes.c_double))]


class Launch(ctypes.Structure):
    _fields_ = [("steps_per_launch", ctypes.c_int32), ("strip_rows", ctypes.c_int32),
                ("strips_per_group", ctypes.c_int32), ("tile", ctypes.c_int32)]

    def as_tuple(self):
        return (self.steps_per_launch, self.strip_rows, self.strips_per_group, self.tile)


class BatchConfig(ctypes.Structure):
    _fields_ = [("steps_per_launch", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("graph_launches", ctypes.c_int32), ("strip_rows", ctypes.c_int32)]

    def as_tuple(self):
        return (self.steps_per_launch, self.blocks_per_cu, self.graph_launches, self.strip_rows)


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class ServerOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("memory_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("check_interval", ctypes.c_int32), ("launch", BatchConfig)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("error", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("steps", ctypes.c_int64), ("residual", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("active", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("node_updates", ctypes.c_int64), ("busy_seconds", ctypes.c_double),
                ("memory_in_use", ctypes.c_size_t), ("memory_high_water", ctypes.c_size_t)]


def _struct_dict(st):
    return {name: getattr(st, name) for name, _ in st._fields_}


class BtrtError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        self.code = code
        super().__init__(f"{where}: {msg} (code {code})")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libbtrt.so (built by paper_1902_09813_amd/build.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python paper_1902_09813_amd/build.py")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 (same soname). Loading
        # torch first makes libbtrt bind to that copy, so device pointers and streams handed
        # over from torch belong to the runtime the library launches on. Without torch the
        # system runtime is used.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        hp = ctypes.c_void_p
        sig = {
            "btrt_validate": ([P(Grid), P(Flux), P(Diff), P(DTerm), P(Source), P(BC), P(Relax), P(Info)], ctypes.c_int),
            "btrt_workspace_size": ([P(Grid), P(Diff), P(Source)], ctypes.c_size_t),
            "btrt_create": ([P(Grid), P(Flux), P(Diff), P(DTerm), P(Source), P(BC), P(Relax), dp, P(hp)], ctypes.c_int),
            "btrt_step": ([hp, ctypes.c_int64], ctypes.c_int),
            "btrt_set_walls": ([hp, dp, ctypes.c_int64], ctypes.c_int),
            "btrt_set_fusion": ([hp, ctypes.c_int32], ctypes.c_int),
            "btrt_set_launch": ([hp, P(Launch)], ctypes.c_int),
            "btrt_get_launch": ([hp, P(Launch)], ctypes.c_int),
            "btrt_tune": ([hp, ctypes.c_int64, P(Launch), P(ctypes.c_int64)], ctypes.c_int),
            "btrt_field": ([hp, dp], ctypes.c_int),
            "btrt_populations": ([hp, dp], ctypes.c_int),
            "btrt_residual": ([hp, dp], ctypes.c_int),
            "btrt_error": ([hp, dp, dp], ctypes.c_int),
            "btrt_solve": ([hp, ctypes.c_double, ctypes.c_int64, P(ctypes.c_int64), dp], ctypes.c_int),
            "btrt_sync": ([hp], ctypes.c_int),
            "btrt_get_info": ([hp, P(Info)], ctypes.c_int),
            "btrt_destroy": ([hp], ctypes.c_int),
            "btrt_checkpoint_size": ([hp, P(ctypes.c_size_t)], ctypes.c_int),
            "btrt_checkpoint": ([hp, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
            "btrt_restore": ([hp, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
            "btrt_batch_create": ([ctypes.c_int32, P(ProblemDesc), ctypes.c_int32, ctypes.c_void_p, P(hp)], ctypes.c_int),
            "btrt_batch_step": ([hp, ctypes.c_int64], ctypes.c_int),
            "btrt_batch_field": ([hp, ctypes.c_int32, dp], ctypes.c_int),
            "btrt_batch_residual": ([hp, dp], ctypes.c_int),
            "btrt_batch_set_config": ([hp, P(BatchConfig)], ctypes.c_int),
            "btrt_batch_get_config": ([hp, P(BatchConfig)], ctypes.c_int),
            "btrt_batch_tune": ([hp, ctypes.c_int64, P(BatchConfig), P(ctypes.c_int64)], ctypes.c_int),
            "btrt_batch_steps": ([hp, P(ctypes.c_int64)], ctypes.c_int),
            "btrt_batch_sync": ([hp], ctypes.c_int),
            "btrt_batch_destroy": ([hp], ctypes.c_int),
            "btrt_server_create": ([P(ServerOpts), P(hp)], ctypes.c_int),
            "btrt_server_submit": ([hp, P(ProblemDesc), ctypes.c_double, ctypes.c_int64, P(ctypes.c_int64)], ctypes.c_int),
            "btrt_server_pump": ([hp, P(ctypes.c_int32), P(ctypes.c_int32)], ctypes.c_int),
            "btrt_server_info": ([hp, ctypes.c_int64, P(RequestInfo)], ctypes.c_int),
            "btrt_server_result": ([hp, ctypes.c_int64, dp], ctypes.c_int),
            "btrt_server_stats": ([hp, P(ServerStats)], ctypes.c_int),
            "btrt_server_clock": ([hp], ctypes.c_double),
            "btrt_server_destroy": ([hp], ctypes.c_int),
            "btrt_solve_static": ([P(Grid), P(Flux), P(Diff), P(DTerm), P(Source), P(BC), P(Relax), dp, ctypes.c_double,
                                   ctypes.c_int64, dp, P(ctypes.c_int64), dp], ctypes.c_int),
            "btrt_strerror": ([ctypes.c_int], ctypes.c_char_p),
            "btrt_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int, where: str) -> None:
    if rc != OK:
        msg = lib().btrt_last_error().decode() or lib().btrt_strerror(rc).decode()
        raise BtrtError(rc, where, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Problem:
    """The arguments of btrt_create (Eq. (1) with D = phi I), as ctypes structures.

    flux_a, flux_b, flux_c, flux_q: B(phi) = a phi + b phi^2/2 + c |phi|^q; A0 = (k11, k12, k22),
    beta: A = A0 (1 + beta phi^2); A0_field: None or an (ny, nx, 3) array of per-node
    (a11, a12, a22) replacing A0; source: None, an (ny, nx) array, ("sin", amp, kx, ky) or
    ("field", array, growth) for S(x, t) = exp(growth t) array(x); src_r, src_p: the source gains
    r phi (1 - |phi|^p); dterm: None (D = phi I) or (g, e, s) for D = (g phi + e |phi|^s) I;
    bc_type/bc_value for sides x-, x+, y-, y+; k0; k2: "hbb" (Eq. (62)), a scalar (K2 = k2 Ihat)
    or four entries.
    """

    def __init__(self, nx: int, ny: int, *, precision: int = F64, flux_a=(0.0, 0.0), flux_b=(0.0, 0.0),
                 A0=(0.0, 0.0, 0.0), beta: float = 0.0, A0_field=None, source=None, bc_type=(PERIODIC,) * 4,
                 bc_value=(0.0,) * 4, k0: float = 1.0, k2=1.0, check_interval: int = 1000, device: int = 0,
                 flux_c=(0.0, 0.0), flux_q: float = 1.0, src_r: float = 0.0, src_p: float = 1.0, dterm=None):
        self.grid = Grid(int(nx), int(ny), int(precision), int(device), None, None, 0)
        self.flux = Flux((ctypes.c_double * 2)(*flux_a), (ctypes.c_double * 2)(*flux_b),
                         (ctypes.c_double * 2)(*flux_c), float(flux_q))
        self._afield = None
        if A0_field is not None:
            self._afield = np.ascontiguousarray(A0_field, dtype=np.float64).reshape(ny, nx, 3)
        self.diff = Diff(float(A0[0]), float(A0[1]), float(A0[2]), float(beta),
                         _dptr(self._afield) if self._afield is not None else None)
        self.dterm = DTerm(D_PHI_I, 1.0, 0.0, 1.0) if dterm is None else DTerm(D_POLY, *(float(v) for v in dterm))
        self._field = None
        if source is None:
            self.source = Source(SRC_NONE, 0.0, 0, 0, None, 0.0, 0.0, 1.0)
        elif isinstance(source, tuple) and source and source[0] == "sin":
            _, amp, kx, ky = source
            self.source = Source(SRC_SIN, float(amp), int(kx), int(ky), None, 0.0, 0.0, 1.0)
        else:
            growth = 0.0
            if isinstance(source, tuple) and source and source[0] == "field":
                _, source, growth = source
            self._field = np.ascontiguousarray(source, dtype=np.float64).reshape(ny, nx)
            self.source = Source(SRC_FIELD, 0.0, 0, 0, _dptr(self._field), float(growth), 0.0, 1.0)
        self.source.r = float(src_r)
        self.source.p = float(src_p)
        self.bc = BC((ctypes.c_int32 * 4)(*bc_type), (ctypes.c_double * 4)(*bc_value))
        if isinstance(k2, str):
            assert k2 == "hbb"
            self.relax = Relax(float(k0), K2_HBB, (ctypes.c_double * 4)(0, 0, 0, 0), int(check_interval))
        else:
            vals = [float(k2)] * 4 if np.isscalar(k2) else [float(v) for v in k2]
            self.relax = Relax(float(k0), K2_VALUE, (ctypes.c_double * 4)(*vals), int(check_interval))

    @property
    def nx(self) -> int:
        return self.grid.nx

    @property
    def ny(self) -> int:
        return self.grid.ny

    def args(self):
        b = ctypes.byref
        return (b(self.grid), b(self.flux), b(self.diff), b(self.dterm), b(self.source), b(self.bc), b(self.relax))

    def validate(self) -> Info:
        """btrt_validate: host-side checks and derived constants; raises BtrtError."""
        info = Info()
        _check(lib().btrt_validate(*self.args(), ctypes.byref(info)), "btrt_validate")
        return info

    def workspace_size(self) -> int:
        return int(lib().btrt_workspace_size(ctypes.byref(self.grid), ctypes.byref(self.diff),
                                             ctypes.byref(self.source)))


class Solver:
    """One btrt handle. ``torch_memory=True`` hands the library a torch-allocated workspace
    and torch's current HIP stream; otherwise the library allocates its own."""

    def __init__(self, problem: Problem, phi0: np.ndarray, torch_memory: bool = False):
        self.problem = problem
        self._workspace = None
        self.torch_stream = None
        if torch_memory:
            import torch  # plumbing only: device memory and the stream

            dev = torch.device("cuda", problem.grid.device)
            nbytes = problem.workspace_size()
            self._workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            problem.grid.workspace = self._workspace.data_ptr()
            problem.grid.workspace_bytes = nbytes
            # torch's current stream, or a torch stream of default priority when that is the
            # legacy null stream (a NULL handle would make the library create its own).
            stream = torch.cuda.current_stream(dev)
            if stream.cuda_stream == 0:
                stream = torch.cuda.Stream(dev)
            self.torch_stream = stream
            problem.grid.stream = stream.cuda_stream
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(problem.ny, problem.nx)
        h = ctypes.c_void_p()
        _check(lib().btrt_create(*problem.args(), _dptr(phi0), ctypes.byref(h)), "btrt_create")
        self.h = h

    # -- calls of include/btrt.h -----------------------------------------------------------
    def step(self, n: int) -> "Solver":
        _check(lib().btrt_step(self.h, int(n)), "btrt_step")
        return self

    def set_walls(self, values: np.ndarray) -> "Solver":
        """btrt_set_walls: Dirichlet values for the next len(values) steps, each row the sides
        sampled every half lattice spacing from corner to corner: x- (2 ny + 1), x+ (2 ny + 1),
        y- (2 nx + 1), y+ (2 nx + 1)."""
        v = np.ascontiguousarray(values, dtype=np.float64)
        P = 4 * (self.problem.nx + self.problem.ny) + 4
        v = v.reshape(-1, P)
        _check(lib().btrt_set_walls(self.h, _dptr(v), int(v.shape[0])), "btrt_set_walls")
        return self

    def set_fusion(self, steps_per_launch: int) -> "Solver":
        _check(lib().btrt_set_fusion(self.h, int(steps_per_launch)), "btrt_set_fusion")
        return self

    def set_launch(self, steps_per_launch: int = 0, strip_rows: int = 0, strips_per_group: int = 0,
                   tile: int = 0) -> "Solver":
        cfg = Launch(int(steps_per_launch), int(strip_rows), int(strips_per_group), int(tile))
        _check(lib().btrt_set_launch(self.h, ctypes.byref(cfg)), "btrt_set_launch")
        return self

    def launch(self) -> tuple:
        """(steps_per_launch, strip_rows, strips_per_group, tile) in force, resolved."""
        cfg = Launch()
        _check(lib().btrt_get_launch(self.h, ctypes.byref(cfg)), "btrt_get_launch")
        return cfg.as_tuple()

    def tune(self, max_steps: int):
        """Times launch shapes on the live state (advancing it) and keeps the fastest; returns
        (shape tuple, steps used)."""
        cfg = Launch()
        used = ctypes.c_int64()
        _check(lib().btrt_tune(self.h, int(max_steps), ctypes.byref(cfg), ctypes.byref(used)), "btrt_tune")
        return cfg.as_tuple(), int(used.value)

    def field(self) -> np.ndarray:
        out = np.empty((self.problem.ny, self.problem.nx), dtype=np.float64)
        _check(lib().btrt_field(self.h, _dptr(out)), "btrt_field")
        return out

    def populations(self) -> np.ndarray:
        out = np.empty((9, self.problem.ny, self.problem.nx), dtype=np.float64)
        _check(lib().btrt_populations(self.h, _dptr(out)), "btrt_populations")
        return out

    def residual(self) -> float:
        out = ctypes.c_double()
        _check(lib().btrt_residual(self.h, ctypes.byref(out)), "btrt_residual")
        return out.value

    def error(self, ref: np.ndarray):
        ref = np.ascontiguousarray(ref, dtype=np.float64).reshape(self.problem.ny, self.problem.nx)
        out = np.empty(3, dtype=np.float64)
        _check(lib().btrt_error(self.h, _dptr(ref), _dptr(out)), "btrt_error")
        return float(out[0]), float(out[1]), float(out[2])

    def solve(self, tol: float, max_steps: int):
        steps = ctypes.c_int64()
        res = ctypes.c_double()
        _check(lib().btrt_solve(self.h, float(tol), int(max_steps), ctypes.byref(steps), ctypes.byref(res)),
               "btrt_solve")
        return int(steps.value), float(res.value)

    def sync(self) -> None:
        _check(lib().btrt_sync(self.h), "btrt_sync")

    def info(self) -> Info:
        info = Info()
        _check(lib().btrt_get_info(self.h, ctypes.byref(info)), "btrt_get_info")
        return info

    def checkpoint(self) -> bytes:
        """btrt_checkpoint: the solver state as bytes."""
        n = ctypes.c_size_t()
        _check(lib().btrt_checkpoint_size(self.h, ctypes.byref(n)), "btrt_checkpoint_size")
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().btrt_checkpoint(self.h, buf, n.value), "btrt_checkpoint")
        return buf.raw

    def restore(self, data: bytes) -> "Solver":
        """btrt_restore: load a checkpoint taken from a handle of the same problem."""
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        _check(lib().btrt_restore(self.h, buf, len(data)), "btrt_restore")
        return self

    def close(self) -> None:
        if getattr(self, "h", None):
            _check(lib().btrt_destroy(self.h), "btrt_destroy")
            self.h = None
        self._workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STATIC_BYTES = 16 << 20  # BTRT_STATIC_BYTES


def solve_static(problem: Problem, phi0: np.ndarray, tol: float, max_steps: int, stream: Optional[int] = None):
    """btrt_solve_static: create, solve and read phi in one call that allocates no device memory
    (the library's fixed array holds every buffer). Returns (phi, steps taken, last residual)."""
    phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(problem.ny, problem.nx)
    g = problem.grid
    grid = Grid(g.nx, g.ny, g.precision, g.device, stream, None, 0)
    out = np.empty((problem.ny, problem.nx), dtype=np.float64)
    steps = ctypes.c_int64()
    res = ctypes.c_double()
    b = ctypes.byref
    _check(lib().btrt_solve_static(b(grid), *problem.args()[1:], _dptr(phi0), float(tol), int(max_steps), _dptr(out),
                                   b(steps), b(res)), "btrt_solve_static")
    return out, int(steps.value), float(res.value)


def problem_from_workload(w, precision: int = F64, device: int = 0, check_interval: int = 1000) -> Problem:
    """btrt_create arguments for a workloads.Workload."""
    return Problem(w.nx, w.ny, precision=precision, flux_a=w.flux_a, flux_b=w.flux_b, A0=w.A0, beta=w.beta,
                   A0_field=getattr(w, "A0_field", None), source=w.source, bc_type=w.bc_type,
                   bc_value=w.bc_value, k0=w.k0, k2=w.k2, check_interval=check_interval, device=device,
                   flux_c=w.flux_c, flux_q=w.flux_q, src_r=w.src_r, src_p=w.src_p, dterm=w.dterm)


def wall_schedule(w, start: int, steps: int) -> np.ndarray:
    """Rows start .. start+steps-1 of a workload's Dirichlet schedule, for Solver.set_walls."""
    return np.stack([np.asarray(w.walls(k), dtype=np.float64) for k in range(start, start + steps)])


class Batch:
    """A btrt batch: independent problems advanced together by one launch per (fused) step.
    ``problems`` is a list of (Problem, phi0) pairs of one precision."""

    def __init__(self, problems, device: int = 0, stream: Optional[int] = None):
        self.problems = [p for p, _ in problems]
        self._phi0 = [np.ascontiguousarray(ph, dtype=np.float64).reshape(p.ny, p.nx) for p, ph in problems]
        arr = (ProblemDesc * len(problems))()
        for k, (p, _) in enumerate(problems):
            arr[k] = ProblemDesc(p.grid, p.flux, p.diff, p.dterm, p.source, p.bc, p.relax, _dptr(self._phi0[k]))
        h = ctypes.c_void_p()
        _check(lib().btrt_batch_create(len(problems), arr, int(device), stream, ctypes.byref(h)), "btrt_batch_create")
        self.h = h
        self.n = len(problems)

    def step(self, n: int) -> "Batch":
        _check(lib().btrt_batch_step(self.h, int(n)), "btrt_batch_step")
        return self

    def field(self, i: int) -> np.ndarray:
        p = self.problems[i]
        out = np.empty((p.ny, p.nx), dtype=np.float64)
        _check(lib().btrt_batch_field(self.h, int(i), _dptr(out)), "btrt_batch_field")
        return out

    def residual(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64)
        _check(lib().btrt_batch_residual(self.h, _dptr(out)), "btrt_batch_residual")
        return out

    def set_config(self, steps_per_launch: int = 2, blocks_per_cu: int = 0, graph_launches: int = 0,
                   strip_rows: int = 0) -> "Batch":
        c = BatchConfig(int(steps_per_launch), int(blocks_per_cu), int(graph_launches), int(strip_rows))
        _check(lib().btrt_batch_set_config(self.h, ctypes.byref(c)), "btrt_batch_set_config")
        return self

    def config(self):
        c = BatchConfig()
        _check(lib().btrt_batch_get_config(self.h, ctypes.byref(c)), "btrt_batch_get_config")
        return c.as_tuple()

    def tune(self, max_steps: int):
        c = BatchConfig()
        used = ctypes.c_int64()
        _check(lib().btrt_batch_tune(self.h, int(max_steps), ctypes.byref(c), ctypes.byref(used)), "btrt_batch_tune")
        return c.as_tuple(), int(used.value)

    def steps(self) -> int:
        v = ctypes.c_int64()
        _check(lib().btrt_batch_steps(self.h, ctypes.byref(v)), "btrt_batch_steps")
        return int(v.value)

    def sync(self) -> None:
        _check(lib().btrt_batch_sync(self.h), "btrt_batch_sync")

    def close(self) -> None:
        if getattr(self, "h", None):
            _check(lib().btrt_batch_destroy(self.h), "btrt_batch_destroy")
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


class Server:
    """A btrt solve server (continuous batching). Requests are (Problem, phi0, tol, max_steps);
    ``pump`` runs one scheduling round."""

    def __init__(self, precision: int = F32, memory_bytes: int = 8 << 30, max_active: int = 64,
                 check_interval: int = 1000, launch=(0, 0, 0, 0), device: int = 0, stream: Optional[int] = None):
        o = ServerOpts(int(precision), int(device), stream, int(memory_bytes), int(max_active), int(check_interval),
                       BatchConfig(*[int(v) for v in launch]))
        h = ctypes.c_void_p()
        _check(lib().btrt_server_create(ctypes.byref(o), ctypes.byref(h)), "btrt_server_create")
        self.h = h
        self._shape = {}

    def submit(self, problem: Problem, phi0: np.ndarray, tol: float, max_steps: int) -> int:
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(problem.ny, problem.nx)
        d = ProblemDesc(problem.grid, problem.flux, problem.diff, problem.dterm, problem.source, problem.bc,
                        problem.relax, _dptr(phi0))
        rid = ctypes.c_int64()
        _check(lib().btrt_server_submit(self.h, ctypes.byref(d), float(tol), int(max_steps), ctypes.byref(rid)),
               "btrt_server_submit")
        self._shape[rid.value] = (problem.ny, problem.nx)
        return int(rid.value)

    def pump(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().btrt_server_pump(self.h, ctypes.byref(a), ctypes.byref(q)), "btrt_server_pump")
        return int(a.value), int(q.value)

    def info(self, rid: int) -> dict:
        st = RequestInfo()
        _check(lib().btrt_server_info(self.h, int(rid), ctypes.byref(st)), "btrt_server_info")
        return _struct_dict(st)

    def result(self, rid: int) -> np.ndarray:
        out = np.empty(self._shape[rid], dtype=np.float64)
        _check(lib().btrt_server_result(self.h, int(rid), _dptr(out)), "btrt_server_result")
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().btrt_server_stats(self.h, ctypes.byref(st)), "btrt_server_stats")
        return _struct_dict(st)

    def clock(self) -> float:
        return float(lib().btrt_server_clock(self.h))

    def close(self) -> None:
        if getattr(self, "h", None):
            _check(lib().btrt_server_destroy(self.h), "btrt_server_destroy")
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
