#!/usr/bin/env python3
"""Smoother throughput benchmark on one MI355X.

Workload: 4096 x 4096 cells, 8 seeded sinkers (eta 1e6 inside, 1 outside,
harmonic nodal eta, rho 1.1 / 1.0), FP64, v = 0 start, p = 0.
Step: 100 sweeps of RAS-Jacobi (tile 64 x 64, halo = k = 4, shift stream
seed 3) through stk_smooth, followed by the energy norm (Sec. 5.4).
Value: GLUP/s = cells x sweeps / step time (HIP events on the stream).

Also reported: every smoother variant at 100 sweeps (Jacobi split, fused,
RBGS, RAS k = 2, 4, 8), the dominant kernel's roofline (RAS outer-iteration
kernel timed per launch with HIP events; algorithmic bytes = one round trip
of vx, vy, eta_c, eta_n, bx, by read and vx, vy written per launch), and the
CPU oracle timed on this host on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


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
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the sharding design is "
              "documented, not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_19061_amd import api, fields, inputs

    dt = torch.float64 if args.dtype == "f64" else torch.float32
    wbytes = 8 if dt == torch.float64 else 4
    n, sweeps, k = args.n, args.sweeps, args.k
    cells = n * n

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
    bx, by = dp.fx, dp.fy
    ax, ay = dp.velocity()
    cx, cy = dp.velocity()
    shifts = api.ras_shifts(3, 64, 64, 64)
    nl = max(sweeps // k, 8)
    for t in range(2):
        api.ras_outer(ctx, dt, dp.grid, ax, ay, dp.eta_c, dp.eta_n, bx, by, cx, cy, 0.7, 64, 64, k, k, *shifts[t])
    torch.cuda.synchronize()
    ev0.record()
    for t in range(nl):
        src, dst = ((ax, ay), (cx, cy)) if t % 2 == 0 else ((cx, cy), (ax, ay))
        api.ras_outer(ctx, dt, dp.grid, *src, dp.eta_c, dp.eta_n, bx, by, *dst, 0.7, 64, 64, k, k,
                      *shifts[t % len(shifts)])
    ev1.record()
    torch.cuda.synchronize()
    launch_ms = ev0.elapsed_time(ev1) / nl
    alg_bytes = 8 * wbytes * cells  # read vx, vy, eta_c, eta_n, bx, by; write vx, vy
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    log(f"[bench] RAS kernel k={k}: {launch_ms:.3f} ms/launch, {achieved:.0f} GB/s effective "
        f"({achieved / HBM_PEAK_GBS:.1%} of HBM peak)")

    # ---- all variants, 100 sweeps each ----
    variants = {}
    if args.variants == "all":
        words = {"jacobi": 12, "jacobi_fused": 8, "rbgs": 22}
        runs = [("jacobi", {}), ("jacobi_fused", {}), ("rbgs", {})]
        runs += [(f"ras_k{kk}", dict(tile_x=64, tile_y=64, k=kk, halo=kk, seed=3)) for kk in (2, 4, 8)]
        for name, kw in runs:
            var = "ras" if name.startswith("ras") else name
            wx, wy = dp.velocity()
            api.smooth(ctx, dt, dp.grid, wx, wy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, sweeps, var, **kw)
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
                              "words_per_lup": w}
            log(f"[bench] {name}: {t_ms:.2f} ms / {sweeps} sweeps, {g:.1f} GLUP/s, {eff:.0f} GB/s effective")

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
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_ras (one RAS outer iteration per launch)",
                     "launch_ms": round(launch_ms, 4), "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "variants": variants,
        "wall_ms_per_step": round(wall / args.steps * 1e3, 4),
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
