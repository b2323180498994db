"""Throughput benchmark of the TL-VLBM hot path on one MI355X.

Workload (the headline configuration): D3Q6x12 lattice, periodic 256^3 grid,
FP32 structure-of-arrays populations, compressible neo-Hookean material
(mu = 1, lambda = 2), F0 = I + 0.05 A (A seeded Gaussian), seeded Fourier
velocity modes of amplitude 1e-3, c = 10 (dt = dx/10), omega = 1.8.  One step
is one pass of the fused pull-stream / recovery / collision kernel over all
16,777,216 nodes (the configuration has no embedded boundary).  Inputs are
resident in HBM before the timed region.

Prints one JSON line:  metric MLUPS (active node updates per second / 1e6),
roofline of the bulk kernel (576 algorithmic bytes per node-step against the
8 TB/s HBM peak, kernel time from HIP events on the library's stream), and the
FP64 CPU oracle timed on a bounded sample of the same recipe.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--n 256]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_NODE_STEP = 576  # 2 * Q * M * 4 bytes, D3Q6x12 FP32
COUNTERS = os.path.join(ROOT, "profiles", "bulk_c3_256_counters.json")
KERNEL_SRC = [os.path.join(ROOT, "paper_2606_20646_amd", "csrc", f) for f in ("bulk.hip", "tl_math.hpp")]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(nodes):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    only if it was taken on the current kernel source and workload."""
    try:
        rec = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash() or rec.get("nodes") != nodes:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(n_sample=128, steps=200):
    """FP64 oracle on the same recipe at n_sample^3 (bounded CPU sample)."""
    from oracle import oracle as O
    import workloads as W
    if not os.path.exists(O.LIB_PATH):
        O.build()
    c = W.config_c3(n_sample)
    s = O.Sim(3, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"])
    s.set_state(c["U0"], dU0=c["dU0"])
    s.step(1)
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    return {"value": round(n_sample ** 3 * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle, same recipe at {n_sample}^3 ({n_sample ** 3} nodes), {steps} steps "
                      f"after 1 untimed step, {dt:.1f} s wall"}


def copy_calibration(gib=1, reps=5):
    """Plain device copy of known size, used to scale the FETCH_SIZE /
    WRITE_SIZE counters of a profiling run to bytes."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_20646_amd import tlvlbm as T

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    N = args.n
    t0 = time.time()
    c = W.config_c3(N)
    log(f"inputs generated in {time.time() - t0:.1f} s")
    g = T.Solver(3, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], precision="fp32",
                 stream=stream.cuda_stream)
    U0 = torch.from_numpy(c["U0"]).cuda()
    dU0 = torch.from_numpy(c["dU0"]).cuda()
    g.set_state(U0, dU0=dU0)
    del U0, dU0
    torch.cuda.synchronize()
    g.step(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record(stream)
    g.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    nodes = N ** 3
    mlups = nodes * args.steps / wall / 1e6
    achieved = BYTES_PER_NODE_STEP * nodes / (kern_ms * 1e-3) / 1e9
    # sanity: the state stays admissible
    Uo = torch.empty((12, nodes), dtype=torch.float64, device="cuda")
    Jo = torch.empty((nodes,), dtype=torch.float64, device="cuda")
    g.moments_into(U=Uo, J=Jo)
    jmin, jmax = float(Jo.min()), float(Jo.max())
    log(f"{args.steps} steps: {wall * 1e3 / args.steps:.3f} ms/step wall, {kern_ms:.3f} ms/step events, "
        f"J in [{jmin:.4f}, {jmax:.4f}]")
    del Uo, Jo
    g.close()
    torch.cuda.synchronize()
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    out = {
        "metric": "D3Q6x12 FP32 MLUPS (fused collide-stream, 256^3 periodic)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; recipe of the 256^3 periodic D3Q6x12 configuration)",
        "config": {"workload": f"D3Q6x12 periodic {N}^3, FP32 SoA populations, neo-Hookean mu=1 lambda=2, "
                               f"F0=I+0.05A, 8 Fourier velocity modes amp 1e-3, c=10, omega=1.8",
                   "nodes": nodes, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(nodes)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
