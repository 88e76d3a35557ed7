"""Build libbtrt.so (the C-ABI library of include/btrt.h) for gfx950 with hipcc, in-tree.

Every source compiles to its own object, in parallel (the sweep kernels of each storage format
and the batched kernels are separate translation units), then one link makes the library.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libbtrt.so")
SOURCES = [os.path.join(CSRC, f) for f in (
    "btrt_sweep_f32.hip", "btrt_sweep_f64.hip", "btrt_sweep_f16dev.hip", "btrt_sweep_bf16dev.hip",
    "btrt_sweep_gen_f64.hip", "btrt_sweep_gen_f32.hip", "btrt_sweep_k0_f64.hip", "btrt_sweep_k0_f32.hip",
    "btrt_sweep_k0_f16dev.hip", "btrt_sweep_k0_bf16dev.hip",
    "btrt_batch_kernels.hip", "btrt_kernels.hip", "btrt3_kernels.hip",
    "btrt_host.cpp", "btrt_group.cpp", "btrt_api.cpp", "btrt_batch.cpp", "btrt_server.cpp", "btrt3_api.cpp",
    "btrt_static.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # Keep the compiler from forming packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # No implicit multiply-add contraction: the kernels write every FMA explicitly, so a node
    # update rounds identically in every kernel (one-step, fused) and on the host.
    "-ffp-contract=off",
    "-Wall",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def _jobs() -> int:
    try:
        return max(1, min(len(SOURCES), len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(len(SOURCES), os.cpu_count() or 1))


def build(verbose: bool = False) -> str:
    """Compile every HIP source into paper_1902_09813_amd/libbtrt.so; returns its path."""
    with tempfile.TemporaryDirectory(prefix="btrt_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(src) + ".o") for src in SOURCES]

        def compile_one(pair):
            src, obj = pair
            cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(max_workers=_jobs()) as pool:
            results = list(pool.map(compile_one, zip(SOURCES, objs)))
        failed = False
        for src, res in zip(SOURCES, results):
            out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l
                            and "not a recognized feature" not in l)
            if out.strip():
                print(out, file=sys.stderr, flush=True)
            if res.returncode != 0:
                print(f"compile failed: {os.path.basename(src)}", file=sys.stderr, flush=True)
                failed = True
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc")
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    sys.exit(0)
