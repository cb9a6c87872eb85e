#!/usr/bin/env python3
"""Smoother throughput benchmark on one MI355X.

Workload: 4096 x 4096 cells, 8 seeded sinkers (eta 1e6 inside, 1 outside,
harmonic nodal eta, rho 1.1 / 1.0), FP64, v = 0 start, p = 0.
Step: 100 sweeps of RAS-Jacobi (tile 64 x 64, halo = k = 4, shift stream
seed 3) through stk_smooth, followed by the energy norm (Sec. 6.4).
Value: GLUP/s = cells x sweeps / step time (HIP events on the stream).

Also reported: every smoother variant at 100 sweeps (Jacobi split, fused,
RBGS, RAS k = 2, 4, 8 with halo k (= Jacobi^k) and with halo 0 (the paper's
thin-overlap form), each with the energy residual reached after 100 sweeps
from 0), the dominant kernel's roofline (RAS outer-iteration
kernel timed per launch with HIP events; algorithmic bytes = one round trip
of vx, vy, eta_c, eta_n, bx, by read and vx, vy written per launch), the CPU
oracle timed on this host on a bounded sample of the same workload, and the
multigrid solves:
  * "solve": 16 sinkers (eta 1e6) over a smooth background with log10(eta)
    uniform on [-2, 4] (contrast up to 1e8), 2048^2 cells, solved to
    E_v <= 1e-8 by FP64 flexible CG preconditioned by an FP64 V-cycle and by
    an FP32 V-cycle (mixed precision, FP64 refinement loop); each result's E_v is
    recomputed from scratch by the library's FP64 energy-norm call, and the two
    results are compared in the energy norm (oracle parity of the solves is
    covered by the tests);
  * "iteration_cost": the same workload at 8192^2, a fixed number of
    iterations in each mode, time per iteration (at 8192^2 and contrast 1e8 a
    solve to 1e-8 does not finish in a few minutes);
  * "batch": 64 independent sinker problems (256^2 .. 2048^2, uneven mix),
    one launch per (level, kernel) across all of them, both modes;
  * "serve": requests with grids drawn from {128, ..., 4096}^2 (contrast
    10^U(2,6)) admitted by HBM footprint under a 64 GB budget and solved by
    continuous batching; per mode a saturation run (all requests at t = 0)
    gives the peak solves/s, then Poisson arrivals at 0.8x that rate give
    solves/s and p50 / p99 latency;
  * "uzawa": the full Stokes system (velocity and pressure) by inexact Uzawa
    cycles (one V(2,2)-cycle and one eta_c-preconditioned pressure step per
    cycle, omega_p = 0.6) from the lithostatic pressure to the global energy
    residual E <= 1e-8, on 8 sinkers of contrast 1e2, plus the pressure
    step's own HBM rate; then the paper's schedule on the smoother workload
    (contrast 1e6): 1000 cycles with viscosity continuation (4 stages of 25
    cycles), reporting the E reached (plain Uzawa converges slowly there).

    python bench.py [--steps K] [--warmup W] [--gpus 1]

For profiling, ``--kernel-only L`` runs just L launches of the RAS
outer-iteration kernel on the 4096^2 workload, followed by two launches of the
streaming probe with the same traffic pattern (6 planes read, 2 written; the
calibration kernel for the HBM byte counters), and prints one JSON line with
their timings.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the streaming RAS kernel (4096^2, FP64, T = 64,
# k = h = 4) from rocprofv3 FETCH_SIZE / WRITE_SIZE, each scaled by what the
# counter reads for the stream probe k_stream6 of known size in the same run
# (profiles/k_ras_stream_4096_f64_k4.md).
# Valid only for the kernel code it was measured on: reported as null once the
# hash of its sources (comments and blank space removed) differs.
RAS_TRAFFIC = {"sources_sha256_16": "6f82aceae28ffd59", "bytes_per_launch": 1.1088e9, "n": 4096, "k": 4, "dtype": "f64"}


def ras_sources_hash():
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("ras_stream.hip", "stencil.hpp", "wave.hpp"):
        with open(os.path.join(ROOT, "paper_2509_19061_amd", "csrc", f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)  # block comments
        src = re.sub(r"//[^\n]*", " ", src)                # line comments
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--sweeps", type=int, default=100)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--variants", default="all", help="'all' or 'none'")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solve-n", type=int, default=2048, help="refinement workload size (0: skip)")
    ap.add_argument("--config3-n", type=int, default=8192, help="refinement workload at full size (0: skip)")
    ap.add_argument("--config3-cap", type=int, default=800, help="iteration cap of the smooth-background FP64 solve")
    ap.add_argument("--config3-cap-f32", type=int, default=2000,
                    help="iteration cap of the smooth-background FP32 V-cycle solve")
    ap.add_argument("--config3-cap-iid", type=int, default=200, help="iteration cap of the i.i.d.-background solves")
    ap.add_argument("--cpu-seconds-1t", type=float, default=10.0, help="CPU oracle sample at 1 thread (s)")
    ap.add_argument("--variants-n", type=int, default=1024, help="smoother-variant solve table size (0: skip)")
    ap.add_argument("--n3d", type=int, default=256, help="3D extension size n^3 (0: skip)")
    ap.add_argument("--batch", default="default", help="'default' (64-instance mix), 'small' or 'none'")
    ap.add_argument("--kernel-only", type=int, default=0, help="profiling mode: L RAS launches + copy calibration")
    ap.add_argument("--serve", type=int, default=16, help="requests per serving run (0: skip)")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95", help="Poisson loads as fractions of saturation")
    ap.add_argument("--uzawa-n", type=int, default=4096, help="Uzawa workload size (0: skip)")
    ap.add_argument("--floor-n", type=int, default=0,
                    help="FP64 floor of E_v: the n^2 contrast-1e6 sinker solve at growing iteration budgets (0: skip)")
    ap.add_argument("--floor-budgets", default="250,500,1000,2000,4000")
    ap.add_argument("--coarsest", type=int, default=32,
                    help="coarsest grid of the solve workloads' hierarchies (solved exactly; the library default is 8)")
    ap.add_argument("--stall-checks", type=int, default=3,
                    help="solves end after this many true-residual checks without halving N_v (0: never)")
    ap.add_argument("--uzawa-parts", default="all", choices=["all", "solve"],
                    help="'solve': only the contrast-1e2 solves (FP64 and FP32 V-cycle) and the pressure step")
    args = ap.parse_args()
    MG_OPTS["coarsest"] = args.coarsest
    MG_OPTS["stall_checks"] = args.stall_checks

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (how it would shard is "
              "documented, not implemented). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    dt = torch.float64 if args.dtype == "f64" else torch.float32
    wbytes = 8 if dt == torch.float64 else 4
    n, sweeps, k = args.n, args.sweeps, args.k
    cells = n * n

    if args.kernel_only:
        return kernel_only(args)

    t0 = time.time()
    prob = inputs.smoother_workload(n, 2)
    log(f"[bench] workload generated in {time.time() - t0:.1f}s")
    ctx = api.Context(0)
    dp = fields.DeviceProblem(prob, dt)
    vx, vy = dp.velocity()
    ras_kw = dict(tile_x=64, tile_y=64, k=k, halo=k, seed=3)

    def step():
        api.smooth(ctx, dt, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, sweeps, "ras", **ras_kw)
        return api.energy_norm(ctx, dt, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record()
    for s in range(args.steps):
        e = step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1) / args.steps
    glups = cells * sweeps / (ms * 1e-3) / 1e9
    log(f"[bench] RAS k={k}: {ms:.3f} ms/step, {glups:.1f} GLUP/s (wall {wall / args.steps * 1e3:.3f} ms/step), "
        f"E = {e[3]:.3e}")

    # ---- dominant kernel: one RAS outer iteration per launch, timed live ----
    # (a context that insists on the streaming kernel, so the timed kernel is known)
    os.environ["STK_RAS_KERNEL"] = "stream"
    kctx = api.Context(0)
    del os.environ["STK_RAS_KERNEL"]
    kernel_name = "k_ras_stream"
    bx, by = dp.fx, dp.fy
    ax, ay = dp.velocity()
    cx, cy = dp.velocity()
    shifts = api.ras_shifts(3, 64, 64, 64)
    nl = max(sweeps // k, 8)
    try:
        api.ras_outer(kctx, dt, dp.grid, ax, ay, dp.eta_c, dp.eta_n, bx, by, cx, cy, 0.7, 64, 64, k, k, *shifts[0])
    except api.StkError:
        kctx.close()
        kctx, kernel_name = ctx, "k_ras"
    for t in range(2):
        api.ras_outer(kctx, dt, dp.grid, ax, ay, dp.eta_c, dp.eta_n, bx, by, cx, cy, 0.7, 64, 64, k, k, *shifts[t])
    torch.cuda.synchronize()
    ev0.record()
    for t in range(nl):
        src, dst = ((ax, ay), (cx, cy)) if t % 2 == 0 else ((cx, cy), (ax, ay))
        api.ras_outer(kctx, dt, dp.grid, *src, dp.eta_c, dp.eta_n, bx, by, *dst, 0.7, 64, 64, k, k,
                      *shifts[t % len(shifts)])
    ev1.record()
    torch.cuda.synchronize()
    launch_ms = ev0.elapsed_time(ev1) / nl
    alg_bytes = 8 * wbytes * cells  # read vx, vy, eta_c, eta_n, bx, by; write vx, vy
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    log(f"[bench] {kernel_name} k={k}: {launch_ms:.3f} ms/launch, {achieved:.0f} GB/s effective "
        f"({achieved / HBM_PEAK_GBS:.1%} of HBM peak)")

    # ---- practical HBM ceiling: a plain streaming pass with the same traffic pattern
    # (6 planes read, 2 written) over the same arrays, timed the same way
    probe_in = [dp.eta_c, dp.eta_n, dp.fx, dp.fy, ax, ay]
    for _ in range(3):
        api.stream_probe(kctx, dt, dp.grid, probe_in, [cx, cy])
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(20):
        api.stream_probe(kctx, dt, dp.grid, probe_in, [cx, cy])
    ev1.record()
    torch.cuda.synchronize()
    probe_ms = ev0.elapsed_time(ev1) / 20
    probe_bytes = 8 * wbytes * (n + 1) * dp.ld
    probe_gbs = probe_bytes / (probe_ms * 1e-3) / 1e9
    ceiling = {"kernel": "k_stream6 (stk_stream_probe: 6 planes read, 2 written, one element per thread)",
               "ms": round(probe_ms, 4), "bytes": probe_bytes, "gbs": round(probe_gbs, 1),
               "frac_of_peak": round(probe_gbs / HBM_PEAK_GBS, 4),
               "ras_alg_rate_over_ceiling": round(achieved / probe_gbs, 4)}
    log(f"[bench] streaming ceiling: {probe_ms:.4f} ms, {probe_gbs:.0f} GB/s ({probe_gbs / HBM_PEAK_GBS:.1%} of peak); "
        f"RAS at {achieved / probe_gbs:.1%} of it")
    fp32 = run_fp32_leg(kctx, prob, sweeps) if args.dtype == "f64" and args.variants == "all" else None

    # ---- all variants, 100 sweeps each ----
    variants = {}
    if args.variants == "all":
        words = {"jacobi": 12, "jacobi_fused": 8, "rbgs": 22}
        runs = [("jacobi", {}), ("jacobi_fused", {}), ("rbgs", {})]
        runs += [(f"ras_k{kk}", dict(tile_x=64, tile_y=64, k=kk, halo=kk, seed=3)) for kk in (2, 4, 8)]
        # the paper's thin-overlap form (halo 0: tile boundaries frozen for k sweeps), a
        # different smoother from Jacobi^k: convergence against k
        runs += [(f"ras_h0_k{kk}", dict(tile_x=64, tile_y=64, k=kk, halo=0, seed=3)) for kk in (2, 4, 8)]
        for name, kw in runs:
            var = "ras" if name.startswith("ras") else name
            wx, wy = dp.velocity()
            api.smooth(ctx, dt, dp.grid, wx, wy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, sweeps, var, **kw)
            e_sweeps = float(api.energy_norm(ctx, dt, dp.grid, wx, wy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy)[3])
            torch.cuda.synchronize()
            reps = 3
            ev0.record()
            for _ in range(reps):
                api.smooth(ctx, dt, dp.grid, wx, wy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, sweeps, var, **kw)
            ev1.record()
            torch.cuda.synchronize()
            t_ms = ev0.elapsed_time(ev1) / reps
            g = cells * sweeps / (t_ms * 1e-3) / 1e9
            w = 8.0 / kw["k"] if var == "ras" else words[var]
            eff = g * w * wbytes
            variants[name] = {"ms_per_100_sweeps": round(t_ms, 3), "glups": round(g, 2),
                              "effective_gbs": round(eff, 1), "frac_hbm": round(eff / HBM_PEAK_GBS, 4),
                              "words_per_lup": w, "e_after_sweeps": e_sweeps}
            log(f"[bench] {name}: {t_ms:.2f} ms / {sweeps} sweeps, {g:.1f} GLUP/s, {eff:.0f} GB/s effective, "
                f"E after {sweeps} sweeps from 0: {e_sweeps:.6e}")
        # residual (r_v = b - M v, r_p = -D v) and energy norm: algorithmic bytes per cell
        # = vx, vy, eta_c, eta_n, fx, fy read (+ rx, ry, rp written for the residual)
        rx, ry, rp = torch.empty_like(dp.fx), torch.empty_like(dp.fy), torch.empty_like(dp.eta_c)
        for name, fn, words_c in (
                ("residual", lambda: api.residual(ctx, dt, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy,
                                                  rx, ry, rp), 9),
                ("energy_norm", lambda: api.energy_norm(ctx, dt, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx,
                                                        dp.fy), 6)):
            fn()
            reps = 10
            _, secs = _timed(lambda: [fn() for _ in range(reps)])
            t_ms = secs * 1e3 / reps
            eff = words_c * wbytes * cells / (t_ms * 1e-3) / 1e9
            variants[name] = {"ms": round(t_ms, 4), "gcells_per_s": round(cells / (t_ms * 1e-3) / 1e9, 2),
                              "effective_gbs": round(eff, 1), "frac_hbm": round(eff / HBM_PEAK_GBS, 4),
                              "words_per_cell": words_c}
            log(f"[bench] {name}: {t_ms:.3f} ms, {eff:.0f} GB/s effective")
        del rx, ry, rp

    # ---- CPU oracle on a bounded sample ----
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import stokes as S
        bxo, byo = S.rhs(prob, prob.fx, prob.fy)
        ox, oy = prob.zeros_v()
        osh = inputs.random_shifts(64, 64, 64, 3)
        it = 0
        c0 = time.perf_counter()
        while True:
            ox, oy = S.ras_outer(prob, bxo, byo, 0.7, 64, 64, k, k, osh[it][0], osh[it][1], ox, oy)
            it += 1
            el = time.perf_counter() - c0
            if el >= args.cpu_seconds or it >= len(osh):
                break
        cpu_glups = cells * k * it / el / 1e9
        cpu = {"value": round(cpu_glups, 4), "unit": "GLUP/s", "cores": S.num_threads(), "kind": "oracle",
               "sample": f"{it} RAS outer iterations (k={k}, T=64, h={k}, FP64) of the {n}x{n} workload "
                         f"= {it * k} of the step's {sweeps} sweeps, {el:.1f} s"}
        log(f"[bench] CPU oracle: {cpu_glups:.3f} GLUP/s on {cpu['cores']} threads ({el:.1f} s)")
        # the same oracle on one thread (the sample is smaller: it runs ~nproc times slower)
        if args.cpu_seconds_1t > 0:
            nthreads = S.num_threads()
            S.set_num_threads(1)
            ox, oy = prob.zeros_v()
            it1 = 0
            c0 = time.perf_counter()
            while True:
                ox, oy = S.ras_outer(prob, bxo, byo, 0.7, 64, 64, k, k, osh[it1][0], osh[it1][1], ox, oy)
                it1 += 1
                el1 = time.perf_counter() - c0
                if el1 >= args.cpu_seconds_1t or it1 >= len(osh):
                    break
            S.set_num_threads(nthreads)
            cpu["one_thread"] = {"value": round(cells * k * it1 / el1 / 1e9, 5), "cores": 1,
                                 "sample": f"{it1} RAS outer iterations (k={k}) of the {n}x{n} workload, {el1:.1f} s"}
            log(f"[bench] CPU oracle, 1 thread: {cpu['one_thread']['value']} GLUP/s ({el1:.1f} s)")

    del vx, vy, ax, ay, cx, cy
    t_ok = (kernel_name == "k_ras_stream" and RAS_TRAFFIC["sources_sha256_16"] == ras_sources_hash()
            and (n, k, args.dtype) == (RAS_TRAFFIC["n"], RAS_TRAFFIC["k"], RAS_TRAFFIC["dtype"]))
    traffic = RAS_TRAFFIC["bytes_per_launch"] if t_ok else None
    solve = run_solves(ctx, args.solve_n) if args.solve_n > 0 else None
    config3 = (run_config3(ctx, args.config3_n, args.config3_cap, args.config3_cap_f32, args.config3_cap_iid)
               if args.config3_n > 0 else None)
    mgvar = run_variants_solve(ctx, args.variants_n) if args.variants_n > 0 else None
    d3 = run_3d(ctx, args.n3d) if args.n3d > 0 else None
    batch = run_batch(ctx, args.batch) if args.batch != "none" else None
    loads = [float(x) for x in args.serve_loads.split(",") if x.strip()]
    served = run_serve(ctx, args.serve, loads=loads) if args.serve > 0 else None
    uz = run_uzawa(ctx, args.uzawa_n, parts=args.uzawa_parts) if args.uzawa_n > 0 else None
    floor = (run_floor(ctx, args.floor_n, [int(x) for x in args.floor_budgets.split(",") if x.strip()])
             if args.floor_n > 0 else None)

    out = {
        "metric": "smoother GLUP/s + % HBM roofline (RAS-Jacobi)",
        "value": round(glups, 2),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"RAS-Jacobi smoother, {n}x{n} cells, 8 seeded sinkers (eta 1e6/1, harmonic "
                               f"nodal eta), tile 64x64, halo=k={k}, {sweeps} sweeps + energy norm per step",
                   "n": n, "sweeps": sweeps, "k": k, "tile": 64, "halo": k},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                     "traffic_over_algorithmic": round(traffic / alg_bytes, 3) if traffic else None,
                     "kernel": f"{kernel_name} (one RAS outer iteration, k={k} sweeps, per launch)",
                     "launch_ms": round(launch_ms, 4), "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "ceiling": ceiling,
        "variants": variants,
        "fp32": fp32,
        "wall_ms_per_step": round(wall / args.steps * 1e3, 4),
        "solve": solve,
        "config3": config3,
        "smoother_variants_solve": mgvar,
        "ext3d": d3,
        "batch": batch,
        "serve": served,
        "uzawa": uz,
        "fp64_floor": floor,
    }
    print(json.dumps(out), flush=True)
    if kctx is not ctx:
        kctx.close()
    ctx.close()


def kernel_only(args):
    """L launches of the RAS outer-iteration kernel, then the copy calibration."""
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    dt = torch.float64 if args.dtype == "f64" else torch.float32
    n, k = args.n, args.k
    prob = inputs.smoother_workload(n, 2)
    os.environ["STK_RAS_KERNEL"] = "stream"
    ctx = api.Context(0)
    del os.environ["STK_RAS_KERNEL"]
    dp = fields.DeviceProblem(prob, dt)
    (ax, ay), (cx, cy) = dp.velocity(), dp.velocity()
    shifts = api.ras_shifts(3, args.kernel_only, 64, 64)

    def launches():
        for t in range(args.kernel_only):
            src, dst = ((ax, ay), (cx, cy)) if t % 2 == 0 else ((cx, cy), (ax, ay))
            api.ras_outer(ctx, dt, dp.grid, *src, dp.eta_c, dp.eta_n, dp.fx, dp.fy, *dst, 0.7, 64, 64, k, k,
                          *shifts[t])

    _, secs = _timed(launches)
    # calibration of the byte counters: the streaming pass with the same traffic pattern
    # (6 planes read, 2 written, whole planes of (n+1) x ld elements), two launches
    probe_in = [dp.eta_c, dp.eta_n, dp.fx, dp.fy, ax, ay]
    _, csecs = _timed(lambda: [api.stream_probe(ctx, dt, dp.grid, probe_in, [cx, cy]) for _ in range(2)])
    w = 8 if dt == torch.float64 else 4
    out = {"kernel": "k_ras_stream", "n": n, "k": k, "launches": args.kernel_only,
           "ms_per_launch": round(secs * 1e3 / args.kernel_only, 4),
           "alg_bytes_per_launch": 8 * w * n * n,
           "calibration_kernel": "k_stream6", "calibration_read_bytes": 6 * w * (n + 1) * dp.ld,
           "calibration_write_bytes": 2 * w * (n + 1) * dp.ld, "calibration_ms": round(csecs * 1e3 / 2, 4)}
    print(json.dumps(out), flush=True)
    ctx.close()


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r = fn()
    e1.record()
    torch.cuda.synchronize()
    return r, e0.elapsed_time(e1) * 1e-3


# Hierarchy options of the solve workloads (set from --coarsest and
# --stall-checks): the coarsest level is solved exactly, and at these
# contrasts a 32^2 coarsest level takes about a third of the iterations of an
# 8^2 one; a solve whose tolerance lies below its FP64 floor ends once
# restarts stop gaining.
MG_OPTS = {"coarsest": 32, "stall_checks": 3}


def run_solves(ctx, n, tol=1e-8, max_iters=4000):
    """FP64 vs FP32-refined solves of the refinement workload."""
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    t0 = time.time()
    prob = inputs.lognormal_background_workload(n)
    log(f"[bench] solve workload {n}^2 generated in {time.time() - t0:.1f}s")
    dp = fields.DeviceProblem(prob, torch.float64)
    m, setup_s = _timed(lambda: api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n, **MG_OPTS))
    info = m.info()
    log(f"[bench] hierarchy: {info['levels']} levels, {info['coarse_unknowns']} coarsest unknowns, "
        f"setup {setup_s:.3f}s")
    res, sols = {}, {}
    for mode in ("f64", "f32_refined"):
        vx, vy = dp.velocity()
        m.solve(mode, vx, vy, None, dp.fx, dp.fy, tol=tol, max_iters=1, allow_notconv=True)  # buffers, plan
        vx, vy = dp.velocity()
        rep, secs = _timed(lambda: m.solve(mode, vx, vy, None, dp.fx, dp.fy, tol=tol, max_iters=max_iters,
                                            allow_notconv=True))
        ev_check = float(api.energy_norm(ctx, torch.float64, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx,
                                         dp.fy)[4])
        sols[mode] = (vx, vy)
        res[mode] = {"seconds": round(secs, 4), "solves_per_s": round(1.0 / secs, 4), "converged": rep["converged"],
                     "iterations": rep["iterations"],
                     "ms_per_iteration": round(secs * 1e3 / max(1, rep["iterations"]), 3),
                     "ev_report": rep["ev"], "ev_recomputed": ev_check}
        log(f"[bench] solve {mode}: {secs:.3f}s, {rep['iterations']} iterations, "
            f"E_v {rep['ev']:.3e} (recomputed {ev_check:.3e})")
    # the FP32-refined result against the FP64 one in the relative energy norm
    # ||d||_A^2 = -<d, M d>, with M d from the library's residual call (f = 0)
    x64, x32 = sols["f64"], sols["f32_refined"]
    d = (x32[0] - x64[0], x32[1] - x64[1])
    zx, zy = torch.zeros_like(dp.fx), torch.zeros_like(dp.fy)
    rx, ry = torch.empty_like(dp.fx), torch.empty_like(dp.fy)

    def energy(v):
        api.residual(ctx, torch.float64, dp.grid, v[0], v[1], None, dp.eta_c, dp.eta_n, zx, zy, rx, ry)
        return float((v[0] * rx).sum() + (v[1] * ry).sum())  # r = -M v, so this is <v, -M v>

    rel = (max(energy(d), 0.0) / energy(x64)) ** 0.5
    del sols, d, x64, x32
    m.close()
    log(f"[bench] refined vs FP64: relative energy-norm difference {rel:.3e}")
    return {"workload": f"{n}x{n} cells, 16 sinkers eta 1e6 over a smooth background with log10(eta) ~ U(-2, 4), "
                        f"V(2,2)-preconditioned flexible CG to E_v <= {tol:g}",
            "n": n, "tol": tol, "levels": info["levels"], "coarsest": MG_OPTS["coarsest"],
            "coarse_unknowns": info["coarse_unknowns"], "setup_s": round(setup_s, 4),
            "f64": res["f64"], "f32_refined": res["f32_refined"],
            "refined_speedup": round(res["f64"]["seconds"] / res["f32_refined"]["seconds"], 3),
            "refined_vs_f64_energy_rel": rel}


def run_uzawa(ctx, n, tol=1e-8, max_cycles=1000, omega_p=0.6, reps=20, parts="all"):
    """Inexact Uzawa solve of the full Stokes system, and the pressure step's rate."""
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    prob = inputs.random_sinkers(n, 8, 2, eta_in=1e2)
    dp = fields.DeviceProblem(prob, torch.float64)
    m = api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n, **MG_OPTS)
    vx, vy, p = dp.velocity() + (dp.field(),)
    api.uzawa_solve(m, dp.grid, vx, vy, p, dp.eta_c, dp.eta_n, dp.fx, dp.fy, allow_notconv=True,
                    max_cycles=1)  # buffers, plan
    vx, vy, p = dp.velocity() + (dp.field(),)

    def solve():
        api.litho_pressure(ctx, dp.grid, dp.fy, p)
        return api.uzawa_solve(m, dp.grid, vx, vy, p, dp.eta_c, dp.eta_n, dp.fx, dp.fy, allow_notconv=True,
                               omega_p=omega_p, tol=tol, max_cycles=max_cycles)

    (rep, hist), secs = _timed(solve)
    e = api.energy_norm(ctx, torch.float64, dp.grid, vx, vy, p, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
    log(f"[bench] uzawa {n}^2: {rep['cycles']} cycles in {secs:.3f}s, E {rep['e']:.3e} (recomputed {e[3]:.3e}), "
        f"E_v {e[4]:.3e}")
    # the same solve with FP32 V-cycles on the FP64 residual
    mvx, mvy, mp = dp.velocity() + (dp.field(),)
    api.uzawa_solve(m, dp.grid, mvx, mvy, mp, dp.eta_c, dp.eta_n, dp.fx, dp.fy, allow_notconv=True, max_cycles=1,
                    mode="f32_refined")  # FP32 buffers, plan
    mvx, mvy, mp = dp.velocity() + (dp.field(),)

    def msolve():
        api.litho_pressure(ctx, dp.grid, dp.fy, mp)
        return api.uzawa_solve(m, dp.grid, mvx, mvy, mp, dp.eta_c, dp.eta_n, dp.fx, dp.fy, allow_notconv=True,
                               omega_p=omega_p, tol=tol, max_cycles=max_cycles, mode="f32_refined")

    (mrep, _), msecs = _timed(msolve)
    me = api.energy_norm(ctx, torch.float64, dp.grid, mvx, mvy, mp, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
    log(f"[bench] uzawa {n}^2 FP32 V-cycle: {mrep['cycles']} cycles in {msecs:.3f}s, E {mrep['e']:.3e} "
        f"(recomputed {me[3]:.3e})")
    mixed = {"seconds": round(msecs, 4), "cycles": mrep["cycles"], "converged": mrep["converged"],
             "ms_per_cycle": round(msecs * 1e3 / max(1, mrep["cycles"]), 3), "e_report": mrep["e"],
             "e_recomputed": float(me[3]), "speedup_vs_f64": round(secs / msecs, 3)}
    del mvx, mvy, mp

    def pressure_steps():
        for _ in range(reps):
            api.uzawa_pressure(ctx, dp.grid, vx, vy, dp.eta_c, omega_p, p)

    pressure_steps()
    _, psecs = _timed(pressure_steps)
    pms = psecs * 1e3 / reps
    words = 7  # update: vx, vy, eta_c, p read, p written; mean removal: p read and written
    gbs = n * n * words * 8 / (pms * 1e-3) / 1e9
    log(f"[bench] uzawa pressure step {n}^2: {pms:.4f} ms, {gbs:.0f} GB/s effective")
    m.close()
    del vx, vy, p, m, dp
    out = {"workload": f"{n}x{n} cells, 8 sinkers (seed 2) eta 1e2 / 1, inexact Uzawa (one V(2,2)-cycle + pressure "
                       f"step, omega_p {omega_p}) from the lithostatic pressure to E <= {tol:g}",
           "n": n, "tol": tol, "seconds": round(secs, 4), "cycles": rep["cycles"], "converged": rep["converged"],
           "ms_per_cycle": round(secs * 1e3 / max(1, rep["cycles"]), 3), "e_start": float(hist[0]),
           "e_report": rep["e"], "e_recomputed": float(e[3]), "ev": float(e[4]),
           "pressure_step": {"ms": round(pms, 4), "words_per_cell": words, "effective_gbs": round(gbs, 1),
                             "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)},
           "f32_refined": mixed}
    if parts == "solve":
        return out

    # the paper's schedule (Sec. 6.2): 1000 cycles, theta stepped 0, 1/4, .., 1 every 25
    # cycles, on the smoother workload (contrast 1e6)
    cprob = inputs.smoother_workload(n)
    cdp = fields.DeviceProblem(cprob, torch.float64)
    cm = api.MG(ctx, cdp.grid, cdp.eta_c, cdp.eta_n, **MG_OPTS)
    cvx, cvy, cp = cdp.velocity() + (cdp.field(),)

    def csolve():
        api.litho_pressure(ctx, cdp.grid, cdp.fy, cp)
        return api.uzawa_solve(cm, cdp.grid, cvx, cvy, cp, cdp.eta_c, cdp.eta_n, cdp.fx, cdp.fy, allow_notconv=True,
                               omega_p=omega_p, tol=tol, max_cycles=1000, stages=4, stage_cycles=25)

    (crep, chist), csecs = _timed(csolve)
    log(f"[bench] uzawa continuation {n}^2 contrast 1e6: {crep['cycles']} cycles in {csecs:.3f}s, E {crep['e']:.3e}")
    # Anderson acceleration (Alg. 1, depth 5) of the same cycles, no continuation
    cvx.zero_()
    cvy.zero_()

    def asolve():
        api.litho_pressure(ctx, cdp.grid, cdp.fy, cp)
        return api.uzawa_anderson(cm, cdp.grid, cvx, cvy, cp, cdp.eta_c, cdp.eta_n, cdp.fx, cdp.fy, depth=5,
                                  allow_notconv=True, omega_p=omega_p, tol=tol, max_cycles=1000)

    (arep, ahist), asecs = _timed(asolve)
    log(f"[bench] uzawa anderson(5) {n}^2 contrast 1e6: {arep['cycles']} steps in {asecs:.3f}s, E {arep['e']:.3e}")
    cvx.zero_()
    cvy.zero_()

    def asolve32():
        api.litho_pressure(ctx, cdp.grid, cdp.fy, cp)
        return api.uzawa_anderson(cm, cdp.grid, cvx, cvy, cp, cdp.eta_c, cdp.eta_n, cdp.fx, cdp.fy, depth=5,
                                  allow_notconv=True, omega_p=omega_p, tol=tol, max_cycles=1000, mode="f32_refined")

    (a32rep, a32hist), a32secs = _timed(asolve32)
    cvx.zero_()
    cvy.zero_()

    def asolve_cont():
        api.litho_pressure(ctx, cdp.grid, cdp.fy, cp)
        return api.uzawa_anderson(cm, cdp.grid, cvx, cvy, cp, cdp.eta_c, cdp.eta_n, cdp.fx, cdp.fy, depth=5,
                                  allow_notconv=True, omega_p=omega_p, tol=tol, max_cycles=1000, stages=4,
                                  stage_cycles=25)

    (acrep, achist), acsecs = _timed(asolve_cont)
    log(f"[bench] uzawa anderson(5) + continuation {n}^2 contrast 1e6: {acrep['cycles']} steps in {acsecs:.3f}s, "
        f"E {acrep['e']:.3e}")
    log(f"[bench] uzawa anderson(5) FP32 V-cycle {n}^2 contrast 1e6: {a32rep['cycles']} steps in {a32secs:.3f}s, "
        f"E {a32rep['e']:.3e}")
    cm.close()
    anderson = {"workload": f"{n}x{n} smoother workload (8 sinkers, eta 1e6 / 1), Anderson depth 5 over the Uzawa "
                           f"cycles, 1000 steps at most",
                "seconds": round(asecs, 4), "steps": arep["cycles"], "converged": arep["converged"],
                "ms_per_step": round(asecs * 1e3 / max(1, arep["cycles"]), 3),
                "e_at": {str(c): float(ahist[c]) for c in (100, 250, 500, 1000) if c < len(ahist)},
                "e_final": arep["e"],
                "f32_refined": {"seconds": round(a32secs, 4), "steps": a32rep["cycles"],
                                "ms_per_step": round(a32secs * 1e3 / max(1, a32rep["cycles"]), 3),
                                "e_final": a32rep["e"]},
                "with_continuation": {"seconds": round(acsecs, 4), "steps": acrep["cycles"],
                                      "ms_per_step": round(acsecs * 1e3 / max(1, acrep["cycles"]), 3),
                                      "e_at": {str(c): float(achist[c]) for c in (100, 250, 500, 1000)
                                               if c < len(achist)},
                                      "e_final": acrep["e"]}}
    cont = {"workload": f"{n}x{n} smoother workload (8 sinkers, eta 1e6 / 1), 4 continuation stages x 25 cycles "
                        f"then the true system, 1000 cycles in all",
            "seconds": round(csecs, 4), "cycles": crep["cycles"], "converged": crep["converged"],
            "ms_per_cycle": round(csecs * 1e3 / max(1, crep["cycles"]), 3), "e_start": float(chist[0]),
            "e_at": {str(c): float(chist[c]) for c in (100, 250, 500, 1000) if c < len(chist)},
            "e_final": crep["e"]}
    out["continuation"] = cont
    out["anderson"] = anderson
    return out


def run_fp32_leg(ctx, prob, sweeps, ks=(2, 4, 8)):
    """The smoother workload in FP32 (fields rounded to FP32): RAS k = 2, 4, 8
    and fused Jacobi at `sweeps` sweeps, and the RAS outer-iteration kernel's
    own roofline at k = 4 (4-byte words)."""
    import torch

    from paper_2509_19061_amd import api, fields

    dt = torch.float32
    dp = fields.DeviceProblem(prob, dt)
    n = prob.nx
    cells = n * n
    out = {"workload": "the smoother workload with every field rounded to FP32", "variants": {}}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    runs = [(f"ras_k{kk}", "ras", dict(tile_x=64, tile_y=64, k=kk, halo=kk, seed=3)) for kk in ks]
    runs.append(("jacobi_fused", "jacobi_fused", {}))
    for name, var, kw in runs:
        vx, vy = dp.velocity()
        api.smooth(ctx, dt, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, sweeps, var, **kw)
        e_sw = float(api.energy_norm(ctx, dt, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy)[3])
        torch.cuda.synchronize()
        reps = 3
        e0.record()
        for _ in range(reps):
            api.smooth(ctx, dt, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, sweeps, var, **kw)
        e1.record()
        torch.cuda.synchronize()
        t_ms = e0.elapsed_time(e1) / reps
        g = cells * sweeps / (t_ms * 1e-3) / 1e9
        w = 8.0 / kw["k"] if var == "ras" else 8
        eff = g * w * 4
        out["variants"][name] = {"ms_per_100_sweeps": round(t_ms, 3), "glups": round(g, 2),
                                 "effective_gbs": round(eff, 1), "frac_hbm": round(eff / HBM_PEAK_GBS, 4),
                                 "words_per_lup": w, "e_after_sweeps": e_sw}
        log(f"[bench] fp32 {name}: {t_ms:.2f} ms / {sweeps} sweeps, {g:.1f} GLUP/s, {eff:.0f} GB/s effective")
        del vx, vy
    # the dominant kernel per launch, k = 4
    (ax, ay), (cx, cy) = dp.velocity(), dp.velocity()
    shifts = api.ras_shifts(3, 64, 64, 64)
    for t in range(2):
        api.ras_outer(ctx, dt, dp.grid, ax, ay, dp.eta_c, dp.eta_n, dp.fx, dp.fy, cx, cy, 0.7, 64, 64, 4, 4, *shifts[t])
    torch.cuda.synchronize()
    nl = 25
    e0.record()
    for t in range(nl):
        src, dst = ((ax, ay), (cx, cy)) if t % 2 == 0 else ((cx, cy), (ax, ay))
        api.ras_outer(ctx, dt, dp.grid, *src, dp.eta_c, dp.eta_n, dp.fx, dp.fy, *dst, 0.7, 64, 64, 4, 4,
                      *shifts[t % len(shifts)])
    e1.record()
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1) / nl
    alg = 8 * 4 * cells
    ach = alg / (launch_ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "kernel": "k_ras_stream<float> (k=4, per launch)",
                       "launch_ms": round(launch_ms, 4), "alg_bytes_per_launch": alg}
    log(f"[bench] fp32 k_ras_stream k=4: {launch_ms:.4f} ms/launch, {ach:.0f} GB/s effective")
    del ax, ay, cx, cy, dp
    return out


def run_variants_solve(ctx, n, tol=1e-8, max_iters=3000):
    """The paper's smoother variants inside the V-cycle (Sec. 6.2, 6.3, 7.3) on
    the refinement workload at n^2, FP64 FCG to E_v <= tol: the finest level
    smoothed by RAS outer iterations of k inner sweeps (8 sweeps per stage, 64 x
    64 tiles) with the full overlap h = k (exactly Jacobi^8) and the paper's
    thin overlap h = 0, k = 1, 2, 4, 8; the mixed smoother (RAS 32 x 32, k = 4,
    h = 0 on the coarse levels); the paper's schedule (5 + 5 sweeps growing by
    2.5 per level, four levels, the last relaxed, mixed smoother)."""
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    prob = inputs.lognormal_background_workload(n)
    dp = fields.DeviceProblem(prob, torch.float64)
    runs = [("default_v22", dict())]
    for kk in (1, 2, 4, 8):
        for h in (kk, 0):
            runs.append((f"fine_k{kk}_h{h}", dict(nu1=8, nu2=8, fine_k=kk, fine_halo=h)))
    runs.append(("mixed_smoother", dict(coarse_smoother="ras", coarse_tile=32, coarse_k=4, coarse_halo=0)))
    runs.append(("paper_schedule", dict(nu1=5, nu2=5, sweep_growth=2.5, max_levels=4, omega=0.5,
                                        coarse_smoother="ras", coarse_tile=32, coarse_k=4, coarse_halo=0)))
    out = {"workload": f"{n}x{n} refinement workload (16 sinkers eta 1e6, smooth log-uniform background), FP64 FCG "
                       f"to E_v <= {tol:g}, at most {max_iters} iterations", "n": n, "runs": {}}
    for name, opts in runs:
        m = api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n, **opts)
        vx, vy = dp.velocity()
        m.solve("f64", vx, vy, None, dp.fx, dp.fy, tol=tol, max_iters=1, allow_notconv=True)  # buffers, plan
        vx, vy = dp.velocity()
        rep, secs = _timed(lambda: m.solve("f64", vx, vy, None, dp.fx, dp.fy, tol=tol, max_iters=max_iters,
                                            allow_notconv=True))
        its = max(1, rep["iterations"])
        out["runs"][name] = {"options": opts, "converged": rep["converged"], "iterations": rep["iterations"],
                             "seconds": round(secs, 4), "ms_per_iteration": round(secs * 1e3 / its, 3),
                             "ev": rep["ev"]}
        log(f"[bench] variants {name}: {rep['iterations']} iterations, {secs:.3f}s, E_v {rep['ev']:.2e}")
        m.close()
        del vx, vy
    return out


def run_3d(ctx, n, sweeps=20):
    """The 3D extension at n^3 cells (4 spherical sinkers, eta 1e4 / 1): fused
    Jacobi and 3D RAS (T = 8, h = k = 2) in FP64 and FP32, GLUP/s and the
    effective HBM rate of the algorithmic bytes (13 words per LUP for Jacobi:
    vx, vy, vz, eta_c, three edge viscosities, bx, by, bz read, vx, vy, vz
    written; 13/k for RAS)."""
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    prob = inputs.random_sinkers3d(n, 4, 8)
    out = {"workload": f"{n}^3 cells, 4 spherical sinkers eta 1e4 / 1, v = 0 start, {sweeps} sweeps", "n": n}
    cells = n ** 3
    for dts, dt in (("f64", torch.float64), ("f32", torch.float32)):
        dp = fields.DeviceProblem3(prob, dt)
        w = 8 if dt == torch.float64 else 4
        res = {}
        for name, var, kw, words in (("jacobi_fused", "jacobi_fused", {}, 13.0),
                                     ("ras_t8_k2", "ras", dict(tile=8, k=2, halo=2, seed=3), 13.0 / 2)):
            v = dp.velocity()
            api.smooth3d(ctx, dt, dp.grid, v, dp.eta, dp.f, 2, var, **kw)
            _, secs = _timed(lambda: api.smooth3d(ctx, dt, dp.grid, v, dp.eta, dp.f, sweeps, var, **kw))
            g = cells * sweeps / secs / 1e9
            eff = g * words * w
            res[name] = {"glups": round(g, 2), "ms_per_sweep": round(secs * 1e3 / sweeps, 4),
                         "effective_gbs": round(eff, 1), "frac_hbm": round(eff / HBM_PEAK_GBS, 4),
                         "words_per_lup": words}
            log(f"[bench] 3d {dts} {name}: {g:.1f} GLUP/s, {eff:.0f} GB/s effective")
            del v
        out[dts] = res
        del dp
        torch.cuda.empty_cache()
    return out


def run_floor(ctx, n, budgets, tol=1e-12):
    """The FP64 floor of the velocity energy residual: FCG solves of the n^2
    smoother workload (8 sinkers, contrast 1e6) from zero with a tolerance
    below what FP64 can reach, stopped at growing iteration budgets.  The
    reported E_v is the true residual recomputed at the stop (the solve
    restarts CG from its iterate whenever the recurrence residual falls below
    tol while the true one does not)."""
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    prob = inputs.smoother_workload(n, 2)
    dp = fields.DeviceProblem(prob, torch.float64)
    m = api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n, **MG_OPTS)
    rows = []
    for b in budgets:
        vx, vy = dp.velocity()
        rep, secs = _timed(lambda: m.solve("f64", vx, vy, None, dp.fx, dp.fy, tol=tol, max_iters=b,
                                            allow_notconv=True))
        ev = float(api.energy_norm(ctx, torch.float64, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy)[4])
        rows.append({"budget": b, "iterations": rep["iterations"], "ev_true": ev, "seconds": round(secs, 3)})
        log(f"[bench] floor {n}^2: budget {b}: E_v {ev:.3e} after {rep['iterations']} iterations ({secs:.2f}s)")
        del vx, vy
    m.close()
    return {"workload": f"{n}x{n} smoother workload (8 sinkers, eta 1e6 / 1), FP64 FCG + V(2,2), tol {tol}",
            "n": n, "runs": rows}


def run_config3(ctx, n, cap, cap_f32, cap_iid, tol=1e-8):
    """The refinement workload at full size: FP64 and FP32-refined solves (FCG
    preconditioned by one V(2,2)-cycle per iteration) of the smooth
    log-uniform background to E_v <= tol within `cap` (FP64) and `cap_f32`
    (FP32 V-cycle) iterations, and of the literal i.i.d. per-cell background
    within `cap_iid` iterations.  The
    FP32-refined result is compared with the FP64 one in the relative energy
    norm (no oracle solve fits at this size: the oracle's parity is tested at
    small sizes)."""
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    out = {"n": n, "tol": tol, "coarsest": MG_OPTS["coarsest"]}
    for name, gen, caps in (("smooth_background", inputs.lognormal_background_workload,
                              {"f64": cap, "f32_refined": cap_f32}),
                             ("iid_background", inputs.iid_log_uniform_workload,
                              {"f64": cap_iid, "f32_refined": cap_iid})):
        t0 = time.time()
        prob = gen(n)
        dp = fields.DeviceProblem(prob, torch.float64)
        del prob
        m, setup_s = _timed(lambda: api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n, **MG_OPTS))
        log(f"[bench] config3 {name} {n}^2 ready in {time.time() - t0:.1f}s (hierarchy {setup_s:.2f}s)")
        res, sols = {}, {}
        for mode in ("f64", "f32_refined"):
            maxit = caps[mode]
            vx, vy = dp.velocity()
            m.solve(mode, vx, vy, None, dp.fx, dp.fy, tol=tol, max_iters=1, allow_notconv=True)  # buffers, plan
            vx, vy = dp.velocity()
            rep, secs = _timed(lambda: m.solve(mode, vx, vy, None, dp.fx, dp.fy, tol=tol, max_iters=maxit,
                                                allow_notconv=True))
            ev = float(api.energy_norm(ctx, torch.float64, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx,
                                       dp.fy)[4])
            its = max(1, rep["iterations"])
            res[mode] = {"converged": rep["converged"], "iterations": rep["iterations"], "cap": maxit,
                         "seconds": round(secs, 3),
                         "ms_per_iteration": round(secs * 1e3 / its, 3), "ev": ev,
                         "rate_per_iteration": round(ev ** (1.0 / its), 5) if ev > 0 else None}
            log(f"[bench] config3 {name} {mode}: {rep['iterations']} iterations in {secs:.2f}s, E_v {ev:.3e}")
            sols[mode] = (vx, vy)
        zx, zy = torch.zeros_like(dp.fx), torch.zeros_like(dp.fy)
        rx, ry = torch.empty_like(dp.fx), torch.empty_like(dp.fy)

        def energy(v):
            api.residual(ctx, torch.float64, dp.grid, v[0], v[1], None, dp.eta_c, dp.eta_n, zx, zy, rx, ry)
            return float((v[0] * rx).sum() + (v[1] * ry).sum())

        x64, x32 = sols["f64"], sols["f32_refined"]
        rel = (max(energy((x32[0] - x64[0], x32[1] - x64[1])), 0.0) / max(energy(x64), 1e-300)) ** 0.5
        res["f32_vs_f64_energy_rel"] = rel
        res["error_reference"] = "the FP64 GPU solve of the same run (no oracle solve at this size)"
        if res["f64"]["converged"] and res["f32_refined"]["converged"]:
            res["refined_speedup"] = round(res["f64"]["seconds"] / res["f32_refined"]["seconds"], 3)
        res["refined_speedup_per_iteration"] = round(res["f64"]["ms_per_iteration"]
                                                     / res["f32_refined"]["ms_per_iteration"], 3)
        res["setup_s"] = round(setup_s, 3)
        out[name] = res
        m.close()
        del sols, x64, x32, zx, zy, rx, ry, dp, m
        torch.cuda.empty_cache()
    out["workload"] = (f"{n}x{n} cells, 16 sinkers eta 1e6 (seed 4); smooth_background: log10(eta) ~ U(-2, 4) as a "
                       f"smooth random field; iid_background: log10(eta) ~ U(-2, 4) i.i.d. per cell (the literal "
                       f"reading); FCG with one V(2,2)-cycle per iteration, FP64 and FP32 V-cycle")
    return out


def run_serve(ctx, count, sizes=(128, 256, 512, 1024, 2048, 4096), budget=64 << 30, loads=(0.5, 0.8, 0.95),
              tol=1e-8, max_iters=1000):
    """Per mode: a saturation run (all requests at t = 0) gives the peak
    solves/s, then Poisson arrivals at each fraction of that rate in `loads`
    give solves/s and p50 / p99 latency.  Requests stop at E_v <= tol or after
    max_iters iterations."""
    import numpy as np

    from paper_2509_19061_amd import inputs, serve

    t0 = time.time()
    base = serve.poisson_requests(count, float("inf"), list(sizes), seed=6)
    payload = {r.rid: inputs.instance_problem(r.n, np.random.default_rng(r.seed)) for r in base}
    log(f"[bench] serve: {count} requests built in {time.time() - t0:.1f}s, sizes "
        + ", ".join(f"{n}:{sum(r.n == n for r in base)}" for n in sizes))
    out = {"workload": f"{count} requests per run, n uniform over {list(sizes)}, sinkers U{{1..8}}, contrast "
                       f"10^U(2,6), E_v <= {tol:g} (at most {max_iters} iterations), HBM budget {budget >> 30} GiB, "
                       f"continuous batching; Poisson loads {list(loads)} x saturation",
           "requests": count, "budget_bytes": budget, "loads": list(loads)}
    for mode in ("f64", "f32_refined"):
        res = {}
        runs = ["saturation"] + [f"poisson_{ld:g}" for ld in loads]
        for run, ld in zip(runs, [None] + list(loads)):
            if ld is None:
                reqs = [serve.Request(r.rid, 0.0, r.n, r.seed, payload[r.rid]) for r in base]
            else:
                rate = ld * res["saturation"]["solves_per_s"]
                arr = serve.poisson_requests(count, rate, [0], seed=7)
                reqs = [serve.Request(r.rid, a.arrival, r.n, r.seed, payload[r.rid]) for r, a in zip(base, arr)]
            be = serve.GpuBackend(ctx, mode, 64, tol=tol, max_iters=max_iters, mg_opts=MG_OPTS)
            summ = serve.Server(be, budget, max_slots=64, iters_per_step=4).run(reqs).summary()
            be.close()
            if ld is not None:
                summ["arrival_rate_per_s"] = round(rate, 4)
                summ["load"] = ld
            res[run] = summ
            log(f"[bench] serve {mode} {run}: {summ['solves_per_s']} solves/s, p50 {summ['latency_p50_s']}s, "
                f"p99 {summ['latency_p99_s']}s, admitted while busy {summ['admitted_while_busy']}, "
                f"max in flight {summ['max_inflight']}, converged "
                f"{sum(v['converged'] for v in summ['by_size'].values())}/{summ['completed']}")
        out[mode] = res
    return out


def run_batch(ctx, which, tol=1e-8, max_iters=3000):
    """The 64-instance uneven mix solved in one batch per mode."""
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    sizes = ((256, 28), (512, 20), (1024, 12), (2048, 4)) if which == "default" else ((128, 6), (256, 4), (512, 2))
    t0 = time.time()
    probs = inputs.batch_mix(5, sizes)
    dps = [fields.DeviceProblem(q, torch.float64) for q in probs]
    mgs = [api.MG(ctx, d.grid, d.eta_c, d.eta_n, **MG_OPTS) for d in dps]
    cells = sum(q.nx * q.ny for q in probs)
    log(f"[bench] batch of {len(probs)} instances ({cells / 1e6:.1f} M cells) ready in {time.time() - t0:.1f}s")
    out = {"workload": f"{len(probs)} sinker problems " + ", ".join(f"{c} x {n}^2" for n, c in sizes)
                       + f", contrast 10^U(2,6), E_v <= {tol:g}", "instances": len(probs), "cells": cells,
           "coarsest": MG_OPTS["coarsest"]}
    for mode in ("f64", "f32_refined"):
        vs = [d.velocity() for d in dps]
        reps, secs = _timed(lambda: api.mg_solve_batch(ctx, mgs, mode, [v[0] for v in vs], [v[1] for v in vs], None,
                                                       [d.fx for d in dps], [d.fy for d in dps], tol=tol,
                                                       max_iters=max_iters, allow_notconv=True))
        its = [r["iterations"] for r in reps]
        out[mode] = {"seconds": round(secs, 4), "solves_per_s": round(len(probs) / secs, 3),
                     "all_converged": all(r["converged"] for r in reps), "max_iterations": max(its),
                     "mean_iterations": round(sum(its) / len(its), 1), "max_ev": max(r["ev"] for r in reps)}
        log(f"[bench] batch {mode}: {secs:.3f}s, {len(probs) / secs:.2f} solves/s, iterations max {max(its)}")
        # the same instances solved one after another with the single-instance call
        seq = 0.0
        same = True
        for q, (d, mm) in enumerate(zip(dps, mgs)):
            wx, wy = d.velocity()
            mm.solve(mode, wx, wy, None, d.fx, d.fy, tol=tol, max_iters=1, allow_notconv=True)  # the handle's plan
            wx.zero_()
            wy.zero_()
            rep, secs1 = _timed(lambda: mm.solve(mode, wx, wy, None, d.fx, d.fy, tol=tol, max_iters=max_iters,
                                                 allow_notconv=True))
            seq += secs1
            same = same and torch.equal(wx, vs[q][0]) and torch.equal(wy, vs[q][1])
            del wx, wy
        out[mode]["sequential_seconds"] = round(seq, 4)
        out[mode]["batch_speedup_vs_sequential"] = round(seq / secs, 3)
        out[mode]["batch_equals_sequential_bitwise"] = bool(same)
        log(f"[bench] batch {mode}: sequential single-instance solves {seq:.3f}s ({seq / secs:.2f}x the batch), "
            f"identical results: {same}")
        del vs
    out["refined_speedup"] = round(out["f64"]["seconds"] / out["f32_refined"]["seconds"], 3)
    for mm in mgs:
        mm.close()
    return out


if __name__ == "__main__":
    main()
