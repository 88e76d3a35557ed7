"""Benchmark of the fused B-TriRT D2Q9 sweep on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one time step of the whole hot path over the grid (pull-stream with bounce-back,
moments, block relaxation, equilibrium/source/correction, reconstruction, phi), plus the
Eq. (64) residual reduction every 1000 steps. The workload is the 4096 x 4096 nonlinear
anisotropic problem in FP64 (the configuration whose working set exceeds the 256 MB
Infinity Cache, so the HBM roofline applies). Inputs are resident in HBM before timing.

Prints one JSON line. ``value`` is MLUPS (node updates per microsecond); ``roofline`` compares
the sweep kernel's algorithmic bytes per launch / its average duration with 8 TB/s;
``cpu_baseline`` times the FP64 CPU oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 flops (FMA) x 2.4 GHz.
FP64_PEAK_TFLOPS = 78.6
# VALU lane-instruction issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (every FP64 VALU
# instruction of a 64-wide wavefront occupies its SIMD for four cycles, and so does every FP32 or
# 16-bit one that is not packed).
FP64_ISSUE_PEAK_T = 39.3
# One node update of the 4096^2 nonlinear workload (k0 = 1, K1 per node, Burgers flux, no source)
# as the collision is written: FP64 flops (an FMA counts two) and FP64 VALU instructions.
FLOPS_PER_UPDATE = 112
FP64_INSTRUCTIONS_PER_UPDATE = 81
BYTES_PER_UPDATE_F64 = 160  # 9 populations + phi read, the same written, per node update
CHECK_INTERVAL = 1000
METRIC = "MLUPS and % HBM roofline, batched/served vs plain; p50/p99 solve latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic.json")
CSRC = os.path.join(ROOT, "paper_1902_09813_amd", "csrc")
KERNEL_SOURCES = ("btrt_internal.h", "btrt_node.h", "btrt_device.h", "btrt_sweep_f64.hip", "btrt_sweep_f32.hip",
                  "btrt_sweep_k0_f64.hip", "btrt_sweep_k0_f32.hip", "btrt_sweep_k0_f16dev.hip",
                  "btrt_sweep_k0_bf16dev.hip", "btrt_sweep_f16dev.hip", "btrt_sweep_bf16dev.hip",
                  "btrt_batch_kernels.hip", "btrt_kernels.hip")


def kernel_hash() -> str:
    """sha256 (first 16 hex digits) over the device-code sources, in a fixed order."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sweep_launches(steps, fusion):
    """Sweep launches btrt_step makes for ``steps`` steps, chunked at every residual check."""
    n = 0
    done = 0
    while done < steps:
        k = min(CHECK_INTERVAL, steps - done)
        n += k // fusion + (1 if k % fusion else 0)
        done += k
    return n


def timed_run(w, precision, steps, warmup, fusion=0, launch=None):
    """Warm up, then time exactly ``steps`` steps with HIP events on the library's stream.

    fusion 0: the warm-up starts with btrt_tune (real steps on the live state, at most 300)
    and the fastest launch shape is kept; 1..4: that many steps per launch, automatic strips.
    launch: a fixed (steps_per_launch, strip_rows, strips_per_group, tile) instead."""
    import torch
    from paper_1902_09813_amd import btrt

    prob = btrt.problem_from_workload(w, precision=precision, check_interval=CHECK_INTERVAL)
    solver = btrt.Solver(prob, w.phi0(), torch_memory=True)  # torch memory + a torch stream
    stream = solver.torch_stream  # the stream every kernel of the solver is launched on
    info = solver.info()
    tuned = 0
    if launch:
        solver.set_launch(*launch)
    elif fusion:
        solver.set_fusion(fusion)
    else:
        _, tuned = solver.tune(900)
    shape = solver.launch()
    fusion = shape[0]
    solver.step(max(0, warmup - tuned))
    solver.sync()
    torch.cuda.synchronize()

    # Events bracket every chunk of sweeps between residual checks, so the sweep's average
    # duration excludes the reductions.
    chunks = []
    done = 0
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    residual = None
    while done < steps:
        k = min(CHECK_INTERVAL, steps - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        solver.step(k)
        b.record(stream)
        chunks.append((a, b, k))
        done += k
        if done % CHECK_INTERVAL == 0:
            residual = solver.residual()  # Eq. (64), part of the step's work
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    sweep_ms = sum(a.elapsed_time(b) for a, b, _ in chunks)
    solver.close()
    nodes = w.nx * w.ny
    return {
        "ms_total": total_ms,
        "wall_s": wall,
        "ms_per_step": total_ms / steps,
        "launches": sweep_launches(steps, fusion),
        "launch_ms_avg": sweep_ms / sweep_launches(steps, fusion),
        "mlups": nodes * steps / (total_ms * 1e-3) / 1e6,
        "bytes_per_node_launch": info.bytes_per_node_launch,
        "nodes": nodes,
        "residual": residual,
        "launch": {"steps_per_launch": shape[0], "strip_rows": shape[1], "strips_per_group": shape[2],
                   "tile": shape[3]},
    }


def timed_run3(w, precision, steps, warmup, launch=None):
    """The D3Q19 solver on a Workload3: HIP events on the stream the library launches on (a torch
    stream handed over through the grid), every launch timed together. launch: a fixed
    (steps_per_launch, z_chunk, tile), else the library's automatic shape."""
    import torch
    from paper_1902_09813_amd import btrt3

    prob = btrt3.problem_from_workload3(w, precision=precision, check_interval=CHECK_INTERVAL)
    stream = torch.cuda.Stream()
    prob.grid.stream = stream.cuda_stream
    solver = btrt3.Solver3(prob, w.phi0())
    if launch:
        solver.set_launch(*launch)
    shape = solver.launch()
    info = solver.info()
    solver.step(warmup)
    solver.sync()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    solver.step(steps)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    solver.close()
    nodes = w.nx * w.ny * w.nz
    k = shape[0]
    launches = steps // k + steps % k
    launch_ms = ms / launches
    bw = info.bytes_per_node_launch * nodes / (launch_ms * 1e-3) / 1e9
    return {"mlups": round(nodes * steps / (ms * 1e-3) / 1e6, 1), "launch_us": round(launch_ms * 1e3, 2),
            "launch": {"steps_per_launch": shape[0], "z_chunk": shape[1], "tile": shape[2]},
            "bytes_per_node_launch": info.bytes_per_node_launch, "achieved_gbs": round(bw, 1),
            "hbm_frac": round(bw / HBM_PEAK_GBS, 4), "steps": steps}


def batched_vs_loop(steps=2600, loop_steps=200, tune_steps=1800):
    """The 256 uneven FP32 instances: one batched launch per fused step (tuned) against a loop
    of plain per-instance launches on one stream. Returns MLUPS of both."""
    import torch
    from paper_1902_09813_amd import btrt
    from paper_1902_09813_amd import workloads as W

    ws = W.c4()
    nodes = sum(w.nx * w.ny for w in ws)
    probs = [(btrt.problem_from_workload(w, precision=btrt.F32), w.phi0()) for w in ws]
    stream = torch.cuda.Stream()
    out = {"instances": len(ws), "nodes": nodes}
    with btrt.Batch(probs, stream=stream.cuda_stream) as b:
        best, used = b.tune(tune_steps)
        b.sync()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        b.step(steps - used)
        e.record(stream)
        b.residual()
        torch.cuda.synchronize()
        ms = a.elapsed_time(e)
        out["batched_mlups"] = round(nodes * (steps - used) / (ms * 1e-3) / 1e6, 1)
        out["batched_config"] = {"steps_per_launch": best[0], "blocks_per_cu": best[1], "graph_launches": best[2],
                                 "strip_rows": best[3]}
    with torch.cuda.stream(stream):
        solvers = [btrt.Solver(btrt.problem_from_workload(w, precision=btrt.F32), ph, torch_memory=True)
                   for w, (_, ph) in zip(ws, probs)]
        for s_ in solvers:
            s_.step(2)
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for s_ in solvers:
            s_.step(loop_steps)
        e.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(e)
        for s_ in solvers:
            s_.close()
    out["loop_mlups"] = round(nodes * loop_steps / (ms * 1e-3) / 1e6, 1)
    out["speedup"] = round(out["batched_mlups"] / out["loop_mlups"], 2)
    return out


def precision_errors(w, steps):
    """phi after ``steps`` steps from phi0 in every storage format (automatic launch shape) against
    the FP64 field of the same run: normwise max, L2-relative and GRE (Eq. (63)) over the whole grid."""
    from paper_1902_09813_amd import btrt

    fields = {}
    for name, prec in (("f64", btrt.F64), ("f32", btrt.F32), ("f16dev", btrt.F16DEV), ("bf16dev", btrt.BF16DEV)):
        with btrt.Solver(btrt.problem_from_workload(w, precision=prec), w.phi0(), torch_memory=True) as s:
            s.step(steps)
            fields[name] = s.field()
    ref = fields.pop("f64")
    den_max, den_l2, den_l1 = np.max(np.abs(ref)), np.sqrt(np.sum(ref * ref)), np.sum(np.abs(ref))
    out = {"steps": steps, "against": "FP64 field of the same run (held to the FP64 oracle at 1e-12 by the tests)"}
    for name, phi in fields.items():
        d = phi - ref
        out[name] = {"max": float(np.max(np.abs(d)) / den_max), "l2": float(np.sqrt(np.sum(d * d)) / den_l2),
                     "gre": float(np.sum(np.abs(d)) / den_l1)}
    return out


def _latency_stats(lat):
    lat = np.sort(np.asarray(lat))
    return round(float(np.percentile(lat, 50)), 3), round(float(np.percentile(lat, 99)), 3)


def plain_requests(reqs):
    """The same arrivals served one request at a time by plain single-handle solves (create, solve
    to the same tolerance, read phi, destroy), in arrival order on one stream."""
    import torch
    from paper_1902_09813_amd import btrt

    lat, updates = [], 0
    start = time.perf_counter()
    for t_arr, w, tol, ms in reqs:
        now = time.perf_counter() - start
        if now < t_arr:
            time.sleep(t_arr - now)
        p = btrt.problem_from_workload(w, precision=btrt.F32, check_interval=CHECK_INTERVAL)
        with btrt.Solver(p, w.phi0()) as s:
            steps, _ = s.solve(tol, ms)
            s.field()
        updates += w.nx * w.ny * steps
        lat.append(time.perf_counter() - start - t_arr)
    end = time.perf_counter() - start
    torch.cuda.synchronize()
    p50, p99 = _latency_stats(lat)
    return {"p50_s": p50, "p99_s": p99, "aggregate_mlups": round(updates / end / 1e6, 1), "wall_s": round(end, 2)}


def served(duration_s=20.0, calib_requests=12, seed=5, rate=None, launch=(0, 0, 0, 0), min_requests=200,
           plain=True):
    """Served solves: Poisson arrivals of FP32 requests (side 64..2048, residual <= 1e-8 or
    50000 steps) into the continuous-batching server. The arrival rate is 0.8 x the rate the
    server sustains on a backlog (calibration run). Time to solution is measured from each
    request's scheduled arrival to its completion, on the server clock."""
    import torch
    from paper_1902_09813_amd import btrt
    from paper_1902_09813_amd import workloads as W

    stream = torch.cuda.Stream()
    opts = dict(precision=btrt.F32, memory_bytes=48 << 30, max_active=128, check_interval=1000,
                launch=launch, stream=stream.cuda_stream)
    sustain = None
    if rate is None:
        # Calibration: a backlog of requests submitted at once.
        calib = W.c5(calib_requests, rate=1.0, seed=seed + 7)
        with btrt.Server(**opts) as srv:
            ids = [srv.submit(btrt.problem_from_workload(w, precision=btrt.F32), w.phi0(), tol, ms)
                   for _, w, tol, ms in calib]
            t0 = srv.clock()
            while any(srv.info(i)["status"] < btrt.REQ_DONE for i in ids):
                srv.pump()
            sustain = calib_requests / (srv.clock() - t0)
        rate = 0.8 * sustain
    n_req = max(min_requests, int(rate * duration_s))
    reqs = W.c5(n_req, rate=rate, seed=seed)
    lat, done_ids = [], []
    with btrt.Server(**opts) as srv:
        start = srv.clock()
        pending = list(reqs)
        sched = {}
        while pending or any(srv.info(i)["status"] < btrt.REQ_DONE for i in sched):
            now = srv.clock() - start
            while pending and pending[0][0] <= now:
                t_arr, w, tol, ms = pending.pop(0)
                rid = srv.submit(btrt.problem_from_workload(w, precision=btrt.F32), w.phi0(), tol, ms)
                sched[rid] = start + t_arr
            active, queued = srv.pump()
            if active == 0 and queued == 0 and pending:
                time.sleep(max(0.0, min(0.05, pending[0][0] - (srv.clock() - start))))
        end = srv.clock()
        st = srv.stats()
        steps = []
        for rid, t_arr in sched.items():
            info = srv.info(rid)
            lat.append(info["t_done"] - t_arr)
            steps.append(info["steps"])
    p50, p99 = _latency_stats(lat)
    out = {
        "requests": n_req,
        "rate_per_s": round(rate, 3),
        "sustained_rate_per_s": round(sustain, 3) if sustain else None,
        "launch": list(launch),
        "p50_s": p50,
        "p99_s": p99,
        "mean_steps": round(float(np.mean(steps)), 1),
        "aggregate_mlups": round(st["node_updates"] / (end - start) / 1e6, 1),
        "wall_s": round(end - start, 2),
        "completed": st["completed"],
        "failed": st["failed"],
        "memory_high_water_gb": round(st["memory_high_water"] / 1e9, 2),
    }
    if plain:
        print(f"[bench] served requests: the same {n_req} arrivals through plain per-request solves", file=sys.stderr,
              flush=True)
        out["plain_loop"] = plain_requests(reqs)
        out["aggregate_speedup"] = round(out["aggregate_mlups"] / out["plain_loop"]["aggregate_mlups"], 2)
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w3, w2, steps3=30, steps2=200, steps3_1=3, steps2_1=20, runs=3):
    """The FP64 oracle as it stands, on the host cores: the median of ``runs`` timed runs of a
    fixed number of steps, each from the same state after one untimed step, with every core
    (OpenMP over rows) and with one thread, on the 4096^2 workload and on the 1024^2 one."""
    from oracle import oracle as O
    from tests._cases import oracle_problem, oracle_source

    def timed(w, nthreads, steps):
        o = O.Oracle(oracle_problem(w), w.phi0(), source=oracle_source(w), nthreads=nthreads)
        o.step(1)
        f0, p0 = o.f.copy(), o.phi_prev.copy()
        times = []
        for _ in range(runs):
            o.f[...] = f0
            o.phi_prev[...] = p0
            t = time.perf_counter()
            o.step(steps)
            times.append(time.perf_counter() - t)
        el = float(np.median(times))
        return round(w.nx * w.ny * steps / el / 1e6, 3), el

    v3, el3 = timed(w3, 0, steps3)
    v2, el2 = timed(w2, 0, steps2)
    v3_1, el3_1 = timed(w3, 1, steps3_1)
    v2_1, el2_1 = timed(w2, 1, steps2_1)
    return {
        "value": v3,
        "unit": "MLUPS",
        "cores": O.threads(),
        "kind": "oracle",
        "sample": (f"{w3.name}: median of {runs} runs of {steps3} steps of the {w3.nx}x{w3.ny} grid after one "
                   f"warm-up step ({el3:.2f} s each)"),
        "value_1thread": v3_1,
        "sample_1thread": f"median of {runs} runs of {steps3_1} steps, one thread ({el3_1:.2f} s each)",
        "c2_value": v2,
        "c2_sample": (f"{w2.name}: median of {runs} runs of {steps2} steps of the {w2.nx}x{w2.ny} grid ({el2:.2f} s "
                      f"each)"),
        "c2_value_1thread": v2_1,
        "c2_sample_1thread": f"median of {runs} runs of {steps2_1} steps, one thread ({el2_1:.2f} s each)",
        "host_cpu": _cpu_model(),
    }


def traffic_key(precision_name, launch):
    return (f"{precision_name}_k{launch['steps_per_launch']}_r{launch['strip_rows']}"
            f"_g{launch['strips_per_group']}_t{launch['tile']}")


def counter_record(precision_name, nodes, launch):
    """The committed rocprofv3 counter figures of one launch shape, or None if the kernel source
    changed since the counters were taken or that shape was not measured on this grid."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256_16") != kernel_hash():
        return None
    ent = rec.get(traffic_key(precision_name, launch))
    if not ent or ent.get("nodes") != nodes:
        return None
    return ent


def traffic_for(precision_name, nodes, launch):
    """HBM bytes per sweep launch (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None."""
    ent = counter_record(precision_name, nodes, launch)
    return None if ent is None else ent.get("bytes_per_launch")


def valu_busy_for(precision_name, nodes, launch):
    """Fraction of SIMD cycles with a VALU instruction in flight (SQ_ACTIVE_INST_VALU x 4 over
    1024 SIMDs x GRBM_GUI_ACTIVE per XCD), or None if not measured for this shape and source."""
    ent = counter_record(precision_name, nodes, launch)
    return None if ent is None else ent.get("valu_busy")


def valu_lanes_for(precision_name, nodes, launch):
    """VALU lane-instructions per node update (SQ_INSTS_VALU x 64 over the launch's updates), or
    None if not measured for this shape and source."""
    ent = counter_record(precision_name, nodes, launch)
    return None if ent is None else ent.get("valu_lane_instructions_per_update")


def roofline_of(r, precision_name):
    """Roofline of the timed sweep kernel. One step per launch moves the whole state every step
    and is bound by HBM: achieved = algorithmic bytes per launch / launch time against 8 TB/s. A
    launch that fuses K steps reads and writes the state once for K node updates per node, so its
    bytes per update fall by K and the arithmetic becomes the limit. FP64 storage: achieved = FP64
    flops of the K updates / launch time against the FP64 vector peak. FP32 and 16-bit storage
    (FP32 arithmetic, issued at the FP64 rate when not packed): achieved = the VALU lane-
    instructions the counter record measured for the shape / launch time against the issue peak
    (HBM as the bound when no record covers the shape). The HBM figures stand beside it."""
    k = r["launch"]["steps_per_launch"]
    t = r["launch_ms_avg"] * 1e-3
    nodes = r["nodes"]
    bytes_per_launch = r["bytes_per_node_launch"] * nodes
    hbm_launch = bytes_per_launch / t / 1e9
    out = {
        "kernel": "sweep_kernel" if k == 1 else ("sweep2_kernel" if r["launch"]["tile"] else "walk_kernel"),
        "traffic": traffic_for(precision_name, nodes, r["launch"]),
        "valu_busy": valu_busy_for(precision_name, nodes, r["launch"]),
        "launch": r["launch"],
        "launch_us_avg": round(t * 1e6, 2),
        "hbm_per_launch": {"achieved": round(hbm_launch, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(hbm_launch / HBM_PEAK_GBS, 4), "bytes_per_launch": bytes_per_launch},
    }
    updates = nodes * k
    lanes = valu_lanes_for(precision_name, nodes, r["launch"]) if k > 1 and precision_name != "f64" else None
    if lanes is not None:
        issue = lanes * updates / t / 1e12
        out.update({"bound": "alu", "achieved": round(issue, 2), "peak": FP64_ISSUE_PEAK_T,
                    "unit": "T lane-instructions/s", "frac": round(issue / FP64_ISSUE_PEAK_T, 4),
                    "valu_lane_instructions_per_update": lanes})
        return out
    if k == 1 or precision_name != "f64":
        out.update({"bound": "hbm", "achieved": round(hbm_launch, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_launch / HBM_PEAK_GBS, 4)})
        return out
    tflops = FLOPS_PER_UPDATE * updates / t / 1e12
    issue = FP64_INSTRUCTIONS_PER_UPDATE * updates / t / 1e12
    out.update({
        "bound": "alu",
        "achieved": round(tflops, 2),
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
        "flops_per_update": FLOPS_PER_UPDATE,
        "fp64_issue": {"instructions_per_update": FP64_INSTRUCTIONS_PER_UPDATE, "achieved": round(issue, 2),
                       "peak": FP64_ISSUE_PEAK_T, "unit": "T lane-instructions/s",
                       "frac": round(issue / FP64_ISSUE_PEAK_T, 4)},
        "per_update_vs_one_step_hbm_roofline": round(BYTES_PER_UPDATE_F64 * updates / t / 1e9 / HBM_PEAK_GBS, 3),
    })
    return out


def copy_probe(nbytes):
    """Device-to-device copy of a known size (calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE)."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", choices=["f64", "f32", "f16dev", "bf16dev"], default="f64")
    ap.add_argument("--fusion", type=int, choices=[0, 1, 2, 3, 4, 5, 6, 7], default=0,
                    help="time steps per sweep launch (0: tuned during the warm-up)")
    ap.add_argument("--launch", default="",
                    help="fixed launch shape steps,rows,group,tile for the main measurement (default: tuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP32 and 1024^2 side measurements")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-requests measurement")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="arrival window of the served measurement (at least 200 requests arrive)")
    ap.add_argument("--serve-requests", type=int, default=200, help="fewest requests of the served measurement")
    ap.add_argument("--no-serve-plain", action="store_true",
                    help="skip the plain per-request baseline of the served measurement")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a device copy of this many bytes")
    ap.add_argument("--d3-launch", default="",
                    help="with --d3-only: fixed D3Q19 launch shape steps,z_chunk,tile (default: automatic)")
    ap.add_argument("--d3-only", action="store_true",
                    help="only the D3Q19 side measurement (256^3 nonlinear periodic box), --steps steps")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the sweep is measured on a single MI355X; "
              "multi-GPU runs are not part of this benchmark.", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    from paper_1902_09813_amd import btrt
    from paper_1902_09813_amd import workloads as W

    if args.d3_only:
        launch3 = tuple(int(v) for v in args.d3_launch.split(",")) if args.d3_launch else None
        w3 = W.d3_nonlinear(256, 256, 256)
        p3 = btrt.F64 if args.precision == "f64" else btrt.F32
        print(json.dumps({"workload": w3.name, "precision": args.precision,
                          **timed_run3(w3, p3, args.steps, args.warmup, launch3)}), flush=True)
        return

    precisions = {"f64": btrt.F64, "f32": btrt.F32, "f16dev": btrt.F16DEV, "bf16dev": btrt.BF16DEV}
    prec = precisions[args.precision]
    w = W.c3()
    print(f"[bench] {w.name} {args.precision}: warmup {args.warmup}, timing {args.steps} steps", file=sys.stderr,
          flush=True)
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    r = timed_run(w, prec, args.steps, args.warmup, args.fusion, launch)
    roofline = roofline_of(r, args.precision)
    extra = {}
    if not args.no_extra:
        for name, other in precisions.items():
            if other == prec:
                continue
            print(f"[bench] side measurement: {w.name} {name}", file=sys.stderr, flush=True)
            r2 = timed_run(w, other, min(args.steps, 2000), 50, args.fusion)
            extra[f"c3_{name}_mlups"] = round(r2["mlups"], 1)
            extra[f"c3_{name}_hbm_frac"] = round(
                r2["bytes_per_node_launch"] * r2["nodes"] / (r2["launch_ms_avg"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        for k in (1, 2, 3, 4, 5, 6, 7):
            print(f"[bench] side measurement: {w.name} {args.precision}, {k} steps per launch", file=sys.stderr,
                  flush=True)
            rk = timed_run(w, prec, min(args.steps, 1000), 20, k)
            extra[f"c3_{args.precision}_fusion{k}_mlups"] = round(rk["mlups"], 1)
            extra[f"c3_{args.precision}_fusion{k}_hbm_frac"] = round(
                rk["bytes_per_node_launch"] * rk["nodes"] / (rk["launch_ms_avg"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        # One step per launch in the other plain format.
        for name, other in (("f64", btrt.F64), ("f32", btrt.F32)):
            if name == args.precision:
                continue  # the fusion1 entry above
            print(f"[bench] side measurement: {w.name} {name}, one step per launch", file=sys.stderr, flush=True)
            rk = timed_run(w, other, min(args.steps, 1000), 20, 1)
            extra[f"c3_{name}_fusion1_mlups"] = round(rk["mlups"], 1)
            extra[f"c3_{name}_fusion1_hbm_frac"] = round(
                rk["bytes_per_node_launch"] * rk["nodes"] / (rk["launch_ms_avg"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        print(f"[bench] side measurement: {w.name} reduced-precision errors after 5000 steps", file=sys.stderr,
              flush=True)
        extra["c3_precision_errors"] = precision_errors(w, 5000)
        w2 = W.c2()
        print(f"[bench] side measurement: {w2.name} f64", file=sys.stderr, flush=True)
        r3 = timed_run(w2, btrt.F64, 2000, 50, args.fusion)
        extra["c2_f64_mlups"] = round(r3["mlups"], 1)
        extra["c2_f64_launch_us"] = round(r3["launch_ms_avg"] * 1e3, 2)
        w3 = W.d3_nonlinear(256, 256, 256)
        for name, p3 in (("f64", btrt.F64), ("f32", btrt.F32)):
            print(f"[bench] side measurement: {w3.name} (D3Q19) {name}", file=sys.stderr, flush=True)
            extra[f"d3q19_256_{name}"] = timed_run3(w3, p3, 200, 20)
        print("[bench] side measurement: 256 batched instances vs per-instance loop (f32)", file=sys.stderr,
              flush=True)
        extra["batched_c4_f32"] = batched_vs_loop()
    if not args.no_serve:
        print("[bench] side measurement: served requests (continuous batching)", file=sys.stderr, flush=True)
        extra["served_c5_f32"] = served(args.serve_seconds, min_requests=args.serve_requests,
                                        plain=not args.no_serve_plain)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, W.c2())

    line = {
        "metric": METRIC,
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == btrt.F64 else "f32",
        "data": "synthetic (seeded 16-Gaussian initial field, lattice units)",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "boundary": "periodic",
                   "flux": "B = 0.025 phi^2 (1, 1)", "diffusion": "A = diag(0.01, 0.005)(1 + phi^2)",
                   "k0": 1.0, "k2": 1.0, "residual_check_interval": CHECK_INTERVAL, "parallelism": "single GPU",
                   "population_storage": args.precision},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
        "residual_at_end": r["residual"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
