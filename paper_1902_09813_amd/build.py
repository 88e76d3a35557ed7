"""Build libbtrt.so (the C-ABI library of include/btrt.h) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libbtrt.so")
SOURCES = [os.path.join(CSRC, f) for f in ("btrt_host.cpp", "btrt_group.cpp", "btrt_api.cpp", "btrt_batch.cpp", "btrt_server.cpp", "btrt_kernels.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # Keep the compiler from forming packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # No implicit multiply-add contraction: the kernels write every FMA explicitly, so a node
    # update rounds identically in every kernel (one-step, two-step) and on the host.
    "-ffp-contract=off",
    "-Wall",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into paper_1902_09813_amd/libbtrt.so; returns its path."""
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
