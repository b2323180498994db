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
8 TB/s HBM peak, kernel time from HIP events on the library's stream), the
FP64 CPU oracle timed on a bounded sample of the same recipe, and the other
two parts of the metric measured in the same run: "adjoint_over_forward"
(the embedded sphere 192^3, 4000 steps, the surface-misfit loss: reverse-mode
time over forward time, with central-difference checks of dL/dmu, dL/dlambda
and an initial-velocity direction) and "batched_speedup" (64 random-hole 2D
instances, 2000 steps: per-instance launches over the batched launch).
--no-extras prints the headline alone.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--n 256]

Other workloads (one JSON line each; not the headline):
    --workload c2   embedded annulus 512^2 (+frame), clamp + traction-free
                    surface, projection every 20 steps, 20000 steps: MLUPS and
                    the L2 distance of u to the radial boundary-value problem
    --workload c4   64 embedded 2D instances: batched launch against
                    per-instance launches of the same kernels
    --workload c5   embedded sphere 192^3 (+frame), Neumann surface: reverse
                    mode (record + backward) over forward time, surface misfit
                    against a target at mu* = 1.3, lambda* = 6
    --workload ellipsoid / shell / annulus / affine
                    the analytic benchmarks end to end (rotated ellipsoid
                    with affine Dirichlet data, N = 320; spherical shell under
                    cavity traction, N = 200; 2D annulus under radial
                    traction, N = 196; 2D affine Dirichlet annulus, N = 384):
                    MLUPS and the relative errors against the exact solutions
    --workload tube the finite tube under end stretch and twist (76 x 76 x 300
                    nodes, 100 000 steps to t = 100): MLUPS, the largest
                    displacement and the Jacobian range
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
KERNEL_SRC = [os.path.join(ROOT, "paper_2606_20646_amd", "csrc", f) for f in ("bulk.hip", "tl_math.hpp", "tl_law.hpp")]


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
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 1000; c2 20000, c4 2000, c5 4000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=None,
                    help="grid cells per axis (c3 256, ellipsoid 320, shell 200)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["c3", "c2", "c4", "c5", "ellipsoid", "shell", "annulus", "affine", "tube"], default="c3")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-fd", action="store_true", help="c5: skip the central-difference checks")
    ap.add_argument("--fd-h", type=float, default=1e-3, help="c5: relative step of the central differences")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the reverse-mode and batched parts of the metric")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "c3" and args.steps is None:
        args.steps = 1000
    if args.workload != "c3":
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        {"c2": bench_c2, "c4": bench_c4, "c5": bench_c5, "ellipsoid": bench_analytic,
         "shell": bench_analytic, "annulus": bench_analytic,
         "affine": bench_analytic, "tube": bench_analytic}[args.workload](args)
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_20646_amd import tlvlbm as T

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    N = args.n or 256
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
        "config": {"workload": f"D3Q6x12 periodic {N}^3, FP32 SoA populations and collision (F and its "
                               f"stress formed in FP64 registers), neo-Hookean mu=1 lambda=2, "
                               f"F0=I+0.05A, 8 Fourier velocity modes amp 1e-3, c=10, omega=1.8",
                   "nodes": nodes, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(nodes)},
        "cpu_baseline": cpu,
    }
    if not args.no_extras:
        # the other two parts of the metric, measured in the same run
        out["adjoint_over_forward"] = c5_measure(4000)
        out["batched_speedup"] = c4_measure(2000)
    print(json.dumps(out), flush=True)


def _common(metric, value, unit, steps, warmup, ms, hib, dtype, workload, extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": hib, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded)", "config": {"workload": workload, "parallelism": "single GPU"}}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_c2(args):
    """Embedded annulus 0.25 <= R <= 0.5 on 512^2 (+frame), inner surface
    displaced radially by 0.05 (sine-squared ramp over T_r = 2), outer surface
    traction free, gamma = 10, projection every 20 steps, 20000 steps."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_20646_amd import tlvlbm as T
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from refsol import radial_bvp
    steps = args.steps or 20000
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    c = W.config_c2(512)
    s = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                 origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"], precision=args.precision,
                 stream=stream.cuda_stream)
    s.set_levelset(c["phi"], c["bid"])
    for bid, bc in c["bcs"].items():
        bc = dict(bc)
        s.set_boundary(bid, bc.pop("type"), **bc)
    s.set_state(c["U0"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = s.stats()
    U, u, J = s.moments()
    act = c["phi"] <= 0
    ref = radial_bvp(2, c["mu"], c["lam"], 0.25, 0.5, r_inner=0.30)
    d = c["X"][:, act] - 0.5
    R = np.linalg.norm(d, axis=0)
    u_ex = (ref["r"](R) - R) * d / R
    err = float(np.linalg.norm(u[:, act] - u_ex) / np.linalg.norm(u_ex))
    nact = int(act.sum())
    _common("embedded annulus MLUPS (active nodes, projection every 20 steps)", round(nact * steps / wall / 1e6, 1),
            "MLUPS", steps, 0, round(wall * 1e3 / steps, 4), True, "f32" if args.precision == "fp32" else "f64",
            f"D2Q4x6 annulus 512^2+frame, {nact} active nodes, {st['cut_links']} cut links, mu=1 lambda=10 "
            f"gamma=10, {args.precision}",
            {"u_L2_error_vs_radial_bvp": err, "time": steps * c["dt"], "cg_iterations": st["cg_iterations"],
             "projections": st["projections"], "J_range": [float(J[act].min()), float(J[act].max())]})


def c4_measure(steps=2000, steps_exact=40):
    """64 instances of the random-hole 2D recipe (64^2 .. 512^2), FP32: the
    batched launch against per-instance launches of the same kernels over
    `steps` steps (the recipe's 2000 by default) with the default projection
    (Jacobi sweeps); beside it, `steps_exact` steps with the exact projection
    (multigrid-preconditioned CG).  Returns the speedup record."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_20646_amd import tlvlbm as T
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    cfgs = [W.config_c4_instance(k) for k in range(64)]
    nodes = sum(int((c["phi"] <= 0).sum()) for c in cfgs)
    log(f"[c4] 64 instances, {nodes} active nodes: inputs in {time.perf_counter() - t0:.1f} s")

    def build(sweeps, mg):
        out = []
        for c in cfgs:
            s = T.Solver(2, c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                         origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"], precision="fp32",
                         stream=stream.cuda_stream, cg_multigrid=mg, proj_sweeps=sweeps)
            s.set_levelset(c["phi"], c["bid"])
            for bid, bc in c["bcs"].items():
                bc = dict(bc)
                s.set_boundary(bid, bc.pop("type"), **bc)
            s.set_state(c["U0"])
            out.append(s)
        return out

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    def compare(sweeps, mg, steps):
        # 20 untimed steps on both paths (first launches, graph capture),
        # then `steps` timed steps holding the same number of projections
        A = build(sweeps, mg)
        T.step_each(A, 20)
        ta = timed(lambda: T.step_each(A, steps))
        B = build(sweeps, mg)
        bt = T.Batch(B, use_graph=True)
        tiles = bt.tiles()
        bt.step(20)
        tb = timed(lambda: bt.step(steps))
        bt.close()
        err = 0.0
        for a, b, c in zip(A, B, cfgs):
            act = c["phi"] <= 0
            Ua, Ub = a.moments()[0][:, act], b.moments()[0][:, act]
            err = max(err, float(np.linalg.norm(Ua[:2] - Ub[:2]) / np.linalg.norm(Ua[:2])),
                      float(np.linalg.norm(Ua[2:] - Ub[2:]) / np.linalg.norm(Ua[2:] - np.eye(2).reshape(-1, 1))))
        for x in A + B:
            x.close()
        return ta, tb, err, tiles

    ta, tb, err, tiles = compare(20, False, steps)
    log(f"[c4] {steps} steps: per-instance {ta:.3f} s, batched {tb:.3f} s")
    tc, te, err_mg, _ = compare(0, True, steps_exact)
    return {"value": round(ta / tb, 3), "unit": "x (per-instance time / batched time)", "steps": steps,
            "workload": f"64 embedded D2Q4x6 instances (random holes, 64^2..512^2), {nodes} active nodes, "
                        f"FP32, projection every 20 steps (20 damped Jacobi sweeps in both paths)",
            "per_instance_s": round(ta, 4), "batched_s": round(tb, 4),
            "per_instance_MLUPS": round(nodes * steps / ta / 1e6, 1),
            "batched_MLUPS": round(nodes * steps / tb / 1e6, 1),
            "max_rel_diff_v_and_F_minus_I": err,
            "tiles": {"width": tiles[0], "order": tiles[1],
                      "ms_per_bulk_launch": {f"order{o}_w{w}": round(v, 4) for (o, w), v in tiles[2].items()}},
            "exact_projection_multigrid_cg": {"steps": steps_exact, "per_instance_s": round(tc, 4),
                                              "batched_s": round(te, 4), "speedup": round(tc / te, 3),
                                              "max_rel_diff_v_and_F_minus_I": err_mg}}


def bench_c4(args):
    r = c4_measure(args.steps or 2000)
    _common("batched speedup over per-instance launches of the same kernels", r["value"], "x", r["steps"], 0,
            round(r["batched_s"] * 1e3 / r["steps"], 4), True, "f32", r["workload"],
            {k: v for k, v in r.items() if k not in ("value", "unit", "steps", "workload")})


def c5_measure(steps=4000, precision="fp32", fd=True, fd_h=1e-3):
    """The differentiation configuration: embedded sphere R = 0.35 on 192^3
    (+frame), traction-free, v0 = 1e-2 Fourier modes.  Loss
    L = 1/2 sum_{surface nodes} |u - u*|^2 after `steps` steps, u* the final
    displacement of a forward run at mu* = 1.3, lambda* = 6 (FP64).  Times the
    forward (tlvlbm_step) and the reverse mode (tlvlbm_adjoint_record +
    tlvlbm_adjoint_backward: forward with checkpoints and tape, recomputation,
    reverse) in `precision`; with fd, checks dL/dmu, dL/dlambda and the
    derivative along a smooth initial-velocity direction (v0 and its
    gradient moved together) against central differences (relative step
    fd_h) of FP64 forward runs.  Inputs stay in HBM."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_20646_amd import tlvlbm as T
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    c = W.config_c5(192)
    rng = np.random.default_rng(77)
    dvh, ddvh = W.fourier_velocity(c["X"], W.fourier_modes(rng, 3), 1e-2)
    log(f"[c5] inputs in {time.perf_counter() - t0:.1f} s")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()  # noqa: E731
    U0d, dU0d, dvd, ddvd = dev(c["U0"]), dev(c["dU0"]), dev(dvh), dev(ddvh)
    act = torch.from_numpy(c["phi"] <= 0).cuda()

    def mk(mu, lam, prec, U0=U0d, dU0=dU0d):
        s = T.Solver(3, c["n"], c["dx"], c["dt"], mu, lam, omega=c["omega"], origin=c["origin"],
                     periodic_mask=0, proj_every=c["proj_every"], precision=prec, stream=stream.cuda_stream)
        s.set_levelset(c["phi"], c["bid"])
        s.set_boundary(1, "neumann")
        torch.cuda.synchronize()  # device inputs written by torch on its own stream
        s.set_state(U0, dU0=dU0)
        return s

    def final_u(s):
        u = torch.empty((3, act.numel()), dtype=torch.float64, device="cuda")
        s.moments_into(u=u)
        return u

    s = mk(1.3, 6.0, "fp64")
    s.step(steps)
    us = final_u(s)
    S = torch.zeros(act.numel(), dtype=torch.bool, device="cuda")
    S[torch.from_numpy(s.links()["node"]).cuda()] = True
    s.close()
    log(f"[c5] target at mu*=1.3, lambda*=6: {steps} steps")

    def loss_of(u):
        return 0.5 * float((((u - us) * S) ** 2).sum())

    s = mk(c["mu"], c["lam"], precision)
    # one untimed reverse run: one-time tables and the device memory of this shape
    s.adjoint_record(steps)
    dLdu = (final_u(s) - us) * S
    torch.cuda.synchronize()
    s.adjoint_backward(None, dLdu, grad_v0=False, grad_u0=False)
    s.set_state(U0d, dU0=dU0d)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t
    L0 = loss_of(final_u(s))
    gv = torch.empty((3, act.numel()), dtype=torch.float64, device="cuda")
    gd = torch.empty((3, 12, act.numel()), dtype=torch.float64, device="cuda")
    s.set_state(U0d, dU0=dU0d)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.adjoint_record(steps)
    torch.cuda.synchronize()
    tr = time.perf_counter() - t
    dLdu = (final_u(s) - us) * S
    torch.cuda.synchronize()
    t = time.perf_counter()
    gm, _, _, _ = s.adjoint_backward(None, dLdu, grad_v0=gv, grad_u0=False, grad_dU0=gd)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    s.close()
    ad_v = float((gv * dvd).sum() + (gd[:, :3] * ddvd).sum())
    log(f"[c5] forward {tf:.3f} s, record {tr:.3f} s, backward {tb:.3f} s")
    out = {"value": round((tr + tb) / tf, 3), "unit": "ratio (reverse mode time / forward time)", "steps": steps,
           "workload": f"D3Q6x12 sphere 192^3+frame, {int(act.sum())} active nodes, traction free, projection "
                       f"every 20 steps, {precision}; L = 1/2 sum over {int(S.sum())} surface nodes of |u - u*|^2, "
                       f"u* from mu*=1.3 lambda*=6",
           "forward_s": round(tf, 4), "record_s": round(tr, 4), "backward_s": round(tb, 4), "loss": L0,
           "grad": {"mu": float(gm[0]), "lambda": float(gm[1]), "v0_direction": ad_v}}
    if fd:
        def L(mu, lam, h=0.0):
            U0, dU0 = U0d, dU0d
            if h:
                U0, dU0 = U0d.clone(), dU0d.clone()
                U0[:3] += h * dvd
                dU0[:, :3] += h * ddvd
            r = mk(mu, lam, "fp64", U0, dU0)
            r.step(steps)
            val = loss_of(final_u(r))
            r.close()
            return val

        mu, lam = c["mu"], c["lam"]
        # central differences at h and h/2; their Richardson combination
        # removes the O(h^2) truncation (the loss follows waves over 4000
        # steps: at h = 1e-3 the truncation alone is ~1e-4 relative)
        fns = {"mu": (lambda e: L(mu * (1 + e), lam), mu),
               "lambda": (lambda e: L(mu, lam * (1 + e)), lam),
               "v0_direction": (lambda e: L(mu, lam, e), 1.0)}
        cd, rich = {}, {}
        for k, (fn, scale) in fns.items():
            d1 = (fn(fd_h) - fn(-fd_h)) / (2 * fd_h * scale)
            d2 = (fn(fd_h / 2) - fn(-fd_h / 2)) / (fd_h * scale)
            cd[k] = d1
            rich[k] = (4 * d2 - d1) / 3
        out["fd_h"] = fd_h
        out["fd_central"] = cd
        out["fd_richardson"] = rich
        out["fd_rel_err"] = {k: abs(out["grad"][k] - v) / abs(v) for k, v in rich.items()}
        out["fd_central_rel_err"] = {k: abs(out["grad"][k] - v) / abs(v) for k, v in cd.items()}
        log(f"[c5] central differences {cd}, Richardson {rich}; relative errors {out['fd_rel_err']}")
    return out


def bench_c5(args):
    r = c5_measure(args.steps or 4000, args.precision, fd=not args.no_fd, fd_h=args.fd_h)
    _common("reverse-mode time / forward time", r["value"], "ratio", r["steps"], 0,
            round((r["record_s"] + r["backward_s"]) * 1e3 / r["steps"], 4), False,
            "f32" if args.precision == "fp32" else "f64", r["workload"],
            {k: v for k, v in r.items() if k not in ("value", "unit", "steps", "workload")})


def _embedded_solver(T, c, precision, stream, dU0=True):
    s = T.Solver(c["D"], c["n"], c["dx"], c["dt"], c["mu"], c["lam"], omega=c["omega"], gamma=c["gamma"],
                 origin=c["origin"], periodic_mask=0, proj_every=c["proj_every"], precision=precision,
                 stream=stream.cuda_stream)
    s.set_levelset(c["phi"], c["bid"])
    for bid, bc in c["bcs"].items():
        bc = dict(bc)
        s.set_boundary(bid, bc.pop("type"), **bc)
    s.set_state(c["U0"], dU0=c.get("dU0") if dU0 else None)
    return s


def bench_analytic(args):
    """The 3D analytic benchmarks end to end: the rotated ellipsoid with affine
    velocity Dirichlet data (default N = 320, 1472 steps to t = 0.46) or the
    spherical shell with ramped cavity traction (default N = 200, 10000 steps
    to t = 5); MLUPS over active nodes and the relative L2 errors against the
    exact affine field or the radial boundary-value problem."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2606_20646_amd import tlvlbm as T
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import refsol
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    N = args.n or {"ellipsoid": 320, "shell": 200, "annulus": 196, "affine": 384, "tube": 100}[args.workload]
    print(f"[bench] {args.workload} N={N} {args.precision}: building inputs", file=sys.stderr, flush=True)
    if args.workload == "ellipsoid":
        c = W.config_ellipsoid(N)
        desc = f"D3Q6x12 rotated ellipsoid {N}^3+frame, affine velocity Dirichlet surface, omega=1.8"
    elif args.workload == "affine":
        c = W.config_affine_annulus(N)
        desc = f"D2Q4x6 affine annulus {N}^2+frame, affine velocity Dirichlet surfaces, omega=2"
    elif args.workload == "tube":
        c = W.config_tube(N)
        desc = (f"D3Q6x12 finite tube {c['n'][0]}x{c['n'][1]}x{c['n'][2]} (dx = 1/{N}), traction-free walls, "
                f"clamped end, stretch 0.5 L and twist 45 deg at the other (half-cosine ramp T_r = 10), gamma=10")
    elif args.workload == "annulus":
        c = W.config_radial_annulus(N)
        desc = (f"D2Q4x6 radial traction annulus {N}^2+frame, clamped inner surface, ramped radial traction, "
                f"gamma=10, projection every 20 steps")
    else:
        c = W.config_shell(N)
        desc = (f"D3Q6x12 spherical shell {N}^3+frame, ramped cavity traction, traction-free outer surface, "
                f"gamma=10, projection every 20 steps")
    steps = args.steps or c["steps"]
    s = _embedded_solver(T, c, args.precision, stream)
    print(f"[bench] {args.workload} N={N}: {steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = s.stats()
    U, u, J = s.moments()
    t = steps * c["dt"]
    if args.workload in ("ellipsoid", "affine"):
        err = refsol.affine_errors(c, U, u, J, t)
    elif args.workload == "tube":
        act = c["phi"] <= 0
        err = {"max_displacement": float(np.linalg.norm(u[:, act], axis=0).max()),
               "J_range": [float(J[act].min()), float(J[act].max())],
               "v_rms": float(np.sqrt((U[:3, act] ** 2).sum(0).mean()))}
    elif args.workload == "annulus":
        ref = refsol.radial_bvp(2, c["mu"], c["lam"], 0.18, 0.42, r_inner=0.18, Pr_outer=1.0)
        err = refsol.radial_errors(c, ref, U, u, J)
    else:
        ref = refsol.radial_bvp(3, c["mu"], c["lam"], 0.20, 0.38, r_inner=0.28)
        err = refsol.radial_errors(c, ref, U, u, J)
    nact = int((c["phi"] <= 0).sum())
    extra = dict(err, time=t, active_nodes=nact, cut_links=st["cut_links"], projections=st["projections"],
                 cg_iterations=st["cg_iterations"], newton_failures=st["newton_failures"])
    _common(f"{args.workload} MLUPS (active nodes, end to end)", round(nact * steps / wall / 1e6, 1), "MLUPS",
            steps, 0, round(wall * 1e3 / steps, 4), True, "f32" if args.precision == "fp32" else "f64",
            f"{desc}, {args.precision}", extra)


if __name__ == "__main__":
    main()
