"""MI355X (gfx950) B-TriRT D2Q9 lattice Boltzmann hot path (arXiv:1902.09813).

The method runs in libbtrt.so (HIP kernels behind the C ABI of include/btrt.h);
``btrt`` is its ctypes binding and ``workloads`` holds the seeded synthetic inputs.
"""
from . import btrt, workloads  # noqa: F401
from .btrt import Problem, Solver, BtrtError, problem_from_workload  # noqa: F401
