"""Serving loop: solve requests arrive over time (Poisson), are admitted by
their HBM footprint under a device budget, and are solved by continuous
batching (``api.Batch``): requests that arrive while others are on the GPU
join the batch as soon as a slot and memory are free, and every step
advances all solves in flight with one launch per (level, kernel).

Admission does not stall the solves in flight: an admitted request's fields
are uploaded and its multigrid hierarchy is built by a setup thread on a
stream of its own (``GpuBackend.prepare``), while the loop keeps stepping the
batch; the request joins the batch at the first step after its setup is done.
Each request keeps its hierarchy on the device from admission to completion.
Latency = completion time - arrival time on the host clock.  The loop itself
(``Server``) is independent of the GPU: it talks to a backend with
``footprint / prepare / ready / join / step / release`` (or a synchronous
``admit``), which the tests replace by CPU fakes to check admission and
scheduling.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    n: int                  # grid n x n cells
    seed: int               # problem seed (instance_problem)
    payload: object = None  # host problem (inputs.Problem), built before the run


@dataclass
class Done:
    rid: int
    n: int
    arrival: float
    admitted: float
    finished: float
    iterations: int
    ev: float
    converged: bool
    inflight_at_admission: int

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class ServeResult:
    done: list = field(default_factory=list)
    rejected: list = field(default_factory=list)
    makespan: float = 0.0
    steps: int = 0
    max_inflight: int = 0
    peak_bytes: int = 0

    def summary(self):
        lat = np.array([d.latency for d in self.done]) if self.done else np.zeros(1)
        joined = sum(1 for d in self.done if d.inflight_at_admission > 0)
        return {"requests": len(self.done) + len(self.rejected), "completed": len(self.done),
                "rejected": len(self.rejected),
                "all_converged": all(d.converged for d in self.done),
                "solves_per_s": round(len(self.done) / self.makespan, 4) if self.makespan > 0 else None,
                "makespan_s": round(self.makespan, 4),
                "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
                "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
                "latency_mean_s": round(float(lat.mean()), 4),
                "admitted_while_busy": joined, "max_inflight": self.max_inflight,
                "peak_bytes": self.peak_bytes, "steps": self.steps, "by_size": self.by_size()}

    def by_size(self):
        out = {}
        for n in sorted({d.n for d in self.done}):
            ds = [d for d in self.done if d.n == n]
            lat = np.array([d.latency for d in ds])
            conv = [d for d in ds if d.converged]
            out[str(n)] = {"completed": len(ds), "converged": len(conv),
                           "mean_iterations": round(float(np.mean([d.iterations for d in ds])), 1),
                           "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
                           "worst_ev": float(max(d.ev for d in ds))}
        return out


def poisson_requests(count, rate, sizes, seed):
    """``count`` requests with exponential inter-arrival times of mean 1/rate
    (rate = inf: all at t = 0) and sizes drawn uniformly from ``sizes``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        if np.isfinite(rate):
            t += float(rng.exponential(1.0 / rate))
        out.append(Request(i, t if np.isfinite(rate) else 0.0, int(rng.choice(sizes)), int(rng.integers(1 << 31))))
    return out


class Server:
    """Admission (FIFO, by footprint under ``budget_bytes``, at most
    ``max_slots`` in flight) + continuous batching over ``backend``."""

    def __init__(self, backend, budget_bytes, max_slots=64, iters_per_step=4, clock=time.perf_counter,
                 sleep=time.sleep):
        self.b = backend
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.iters = int(iters_per_step)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests):
        res = ServeResult()
        queue = collections.deque(sorted(requests, key=lambda r: r.arrival))
        pending = collections.deque()
        preparing = collections.deque()  # (request, token, bytes, in flight when admitted), FIFO
        inflight = {}  # slot -> (request, handle, bytes, joined, in flight when admitted)
        used = 0
        asynchronous = hasattr(self.b, "prepare")
        t0 = self.clock()
        while queue or pending or preparing or inflight:
            now = self.clock() - t0
            while queue and queue[0].arrival <= now:
                pending.append(queue.popleft())
            # admission: memory and a slot are reserved now; the setup runs beside the batch
            while pending and len(inflight) + len(preparing) < self.max_slots:
                r = pending[0]
                need = self.b.footprint(r)
                if need > self.budget:  # can never fit
                    res.rejected.append(pending.popleft().rid)
                    continue
                if used + need > self.budget:
                    break
                pending.popleft()
                busy = len(inflight) + len(preparing)
                used += need
                res.peak_bytes = max(res.peak_bytes, used)
                if asynchronous:
                    preparing.append((r, self.b.prepare(r), need, busy))
                else:
                    handle, slot = self.b.admit(r)
                    inflight[slot] = (r, handle, need, self.clock() - t0, busy)
            # requests whose setup is done join the batch (in admission order)
            while preparing and (self.b.ready(preparing[0][1]) or not inflight):
                r, token, need, busy = preparing.popleft()
                handle, slot = self.b.join(token)  # waits for the setup if the batch is idle
                inflight[slot] = (r, handle, need, self.clock() - t0, busy)
            res.max_inflight = max(res.max_inflight, len(inflight))
            if not inflight:
                if queue and not preparing:
                    self.sleep(max(0.0, queue[0].arrival - (self.clock() - t0)))
                continue
            finished = self.b.step(self.iters)
            res.steps += 1
            now = self.clock() - t0
            for slot, rep in finished:
                r, handle, need, admitted, busy = inflight.pop(slot)
                self.b.release(handle)
                used -= need
                res.done.append(Done(r.rid, r.n, r.arrival, admitted, now, rep["iterations"], rep["ev"],
                                     rep["converged"], busy))
        res.makespan = self.clock() - t0
        return res


class GpuBackend:
    """Requests solved on the GPU.  ``prepare`` hands the request to a setup
    thread, which uploads its fields and builds its hierarchy on a setup
    stream and context of its own, then moves the hierarchy to the serving
    context (``MG.bind``, which drains the setup stream); ``join`` adds it to
    the one ``api.Batch`` that the serving loop steps."""

    def __init__(self, ctx, mode, max_slots, tol=1e-8, max_iters=3000, keep_results=False, mg_opts=None):
        from concurrent.futures import ThreadPoolExecutor

        import torch

        from . import api, fields
        self.api, self.fields, self.torch = api, fields, torch
        self.ctx, self.mode, self.tol, self.max_iters = ctx, mode, tol, max_iters
        self.mg_opts = dict(mg_opts or {})  # hierarchy options of every request (api.MG keywords)
        self.batch = api.Batch(ctx, mode, max_slots)
        self.results = {} if keep_results else None  # rid -> (vx, vy) on the host
        self.setup_stream = torch.cuda.Stream(device=ctx.device)  # default priority
        self.setup_ctx = api.Context(ctx.device, stream=self.setup_stream)
        self.serve_stream = torch.cuda.current_stream(ctx.device)
        self.pool = ThreadPoolExecutor(max_workers=1)

    def footprint(self, r):
        p = r.payload
        ld = self.fields.pad_ld(p.nx)
        g = self.api.Grid(p.nx, p.ny, ld, p.dx, p.dy)
        return self.api.mg_footprint(g, self.mode, **self.mg_opts) + 6 * (p.ny + 1) * ld * 8  # + fields

    def _setup(self, r):
        torch = self.torch
        with torch.cuda.stream(self.setup_stream):
            dp = self.fields.DeviceProblem(r.payload, torch.float64)
            vx, vy = dp.velocity()
        mg = self.api.MG(self.setup_ctx, dp.grid, dp.eta_c, dp.eta_n, **self.mg_opts)
        mg.bind(self.ctx, self.mode)  # the setup stream is drained here
        for t in (dp.eta_c, dp.eta_n, dp.fx, dp.fy, vx, vy):
            t.record_stream(self.serve_stream)  # used by the serving stream from now on
        return (r.rid, dp, mg, vx, vy)

    def prepare(self, r):
        return self.pool.submit(self._setup, r)

    def ready(self, token):
        return token.done()

    def join(self, token):
        handle = token.result()
        rid, dp, mg, vx, vy = handle
        slot = self.batch.add(mg, vx, vy, None, dp.fx, dp.fy, tol=self.tol, max_iters=self.max_iters)
        return handle, slot

    def admit(self, r):
        """Synchronous admission (setup on the serving stream)."""
        dp = self.fields.DeviceProblem(r.payload, self.torch.float64)
        mg = self.api.MG(self.ctx, dp.grid, dp.eta_c, dp.eta_n)
        vx, vy = dp.velocity()
        slot = self.batch.add(mg, vx, vy, None, dp.fx, dp.fy, tol=self.tol, max_iters=self.max_iters)
        return (r.rid, dp, mg, vx, vy), slot

    def step(self, iters):
        return self.batch.step(iters)

    def release(self, handle):
        rid, dp, mg, vx, vy = handle
        if self.results is not None:
            self.results[rid] = (dp.get_vx(vx), dp.get_vy(vy))
        mg.close()

    def close(self):
        self.pool.shutdown(wait=True)
        self.batch.close()
        self.setup_ctx.close()
