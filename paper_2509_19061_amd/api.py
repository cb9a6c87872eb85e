"""Python face of the stk C ABI (same call names, torch tensors for memory).

Arguments are device tensors (or raw device pointers as ints); this module
only checks and marshals them.  See ``include/stk.h`` for the semantics.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref

import numpy as np
import torch

from . import _lib as L
from ._lib import (EHIP, EINVAL, ENOMEM, ENONFINITE, ENOTCONV, EUNSUPPORTED, F32, F64, JACOBI, JACOBI_FUSED, OK,
                   RAS_JACOBI, RBGS, SOLVE_F32_REFINED, SOLVE_F64, VARIANTS, Grid, MgOpts, Report, SmoothOpts,
                   StkError, check)

__all__ = ["Context", "Grid", "SmoothOpts", "StkError", "smooth", "ras_outer", "residual", "energy_norm", "ras_shifts",
           "smooth_opts", "energy_norm_noalloc", "stream_probe", "smooth3d", "ras_outer3d", "residual3d",
           "energy_norm3d", "smooth3d_opts", "F64", "F32", "JACOBI", "JACOBI_FUSED", "RAS_JACOBI", "RBGS", "VARIANTS", "OK", "EINVAL",
           "ENOMEM", "EHIP", "ENOTCONV", "ENONFINITE", "EUNSUPPORTED", "dtype_code", "torch_dtype", "MG", "mg_opts",
           "mg_footprint", "mg_solve_batch", "SOLVE_F64", "SOLVE_F32_REFINED", "MODES", "Batch", "uzawa_opts",
           "litho_pressure", "uzawa_pressure", "uzawa_solve", "uzawa_anderson"]

MODES = {"f64": SOLVE_F64, "f32_refined": SOLVE_F32_REFINED}


def dtype_code(dt):
    if dt in (F64, "f64", torch.float64, np.float64):
        return F64
    if dt in (F32, "f32", torch.float32, np.float32):
        return F32
    raise ValueError(f"unsupported dtype {dt!r}")


def torch_dtype(dt):
    return torch.float64 if dtype_code(dt) == F64 else torch.float32


def _ptr(t, dt=None):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"expected a device tensor, got {type(t)}")
    if not t.is_cuda:
        raise ValueError("stk takes device tensors (no CPU path)")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dt is not None and t.dtype != torch_dtype(dt):
        raise ValueError(f"tensor dtype {t.dtype} does not match {dt}")
    return t.data_ptr()


# Live handles, released at interpreter exit while the HIP runtime is still up
# (a destructor that ran during finalisation would call into a torn-down runtime).
_LIVE_CONTEXTS = weakref.WeakSet()


def _close_all():
    for c in list(_LIVE_CONTEXTS):
        try:
            c.close()
        except Exception:
            pass


atexit.register(_close_all)


class Context:
    """stk_ctx bound to a device and a HIP stream (default: torch's current).

    Closing a context first closes the multigrid handles built on it."""

    def __init__(self, device: int = 0, stream=None):
        self.device = device
        self.handle = C.c_void_p()
        self._mgs = weakref.WeakSet()
        self._batches = weakref.WeakSet()
        s = stream if stream is not None else torch.cuda.current_stream(device)
        sp = s.cuda_stream if hasattr(s, "cuda_stream") else s
        check(L.lib.stk_ctx_create(C.byref(self.handle), device, C.c_void_p(sp)))
        _LIVE_CONTEXTS.add(self)

    def set_stream(self, stream):
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        check(L.lib.stk_ctx_set_stream(self.handle, C.c_void_p(sp)))

    def sync(self):
        check(L.lib.stk_ctx_sync(self.handle))

    def scratch_bytes(self):
        n = C.c_size_t()
        check(L.lib.stk_ctx_scratch_bytes(self.handle, C.byref(n)))
        return n.value

    def close(self):
        for b in list(self._batches):
            b.close()
        for m in list(self._mgs):
            m.close()
        if self.handle:
            L.lib.stk_ctx_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def smooth_opts(omega=0.0, tile_x=64, tile_y=64, halo=-1, k=4, shifts=None, seed=0, last_partial=True):
    """Returns (SmoothOpts, keepalive); ``shifts`` is an (n_outer, 2) int array."""
    o = SmoothOpts()
    L.lib.stk_smooth_opts_default(C.byref(o))
    o.omega, o.tile_x, o.tile_y, o.halo, o.k = float(omega), int(tile_x), int(tile_y), int(halo), int(k)
    o.seed, o.last_partial = int(seed), int(bool(last_partial))
    keep = None
    if shifts is not None:
        keep = np.ascontiguousarray(np.asarray(shifts, dtype=np.int32).reshape(-1))
        o.shifts = keep.ctypes.data_as(C.POINTER(C.c_int32))
    return o, keep


def smooth(ctx, dt, grid, vx, vy, p, eta_c, eta_n, fx, fy, sweeps, variant, opts=None, **kw):
    dt = dtype_code(dt)
    if isinstance(variant, str):
        variant = VARIANTS[variant]
    keep = None
    if opts is None and kw:
        opts, keep = smooth_opts(**kw)
    check(L.lib.stk_smooth(ctx.handle, dt, C.byref(grid), _ptr(vx, dt), _ptr(vy, dt), _ptr(p, dt), _ptr(eta_c, dt),
                           _ptr(eta_n, dt), _ptr(fx, dt), _ptr(fy, dt), int(sweeps), int(variant),
                           C.byref(opts) if opts is not None else None))
    del keep


def ras_outer(ctx, dt, grid, vx, vy, eta_c, eta_n, bx, by, ox, oy, omega=0.7, tile_x=64, tile_y=64, halo=4, kt=4,
              sx=0, sy=0):
    dt = dtype_code(dt)
    check(L.lib.stk_ras_outer(ctx.handle, dt, C.byref(grid), _ptr(vx, dt), _ptr(vy, dt), _ptr(eta_c, dt),
                              _ptr(eta_n, dt), _ptr(bx, dt), _ptr(by, dt), _ptr(ox, dt), _ptr(oy, dt), float(omega),
                              int(tile_x), int(tile_y), int(halo), int(kt), int(sx), int(sy)))


def residual(ctx, dt, grid, vx, vy, p, eta_c, eta_n, fx, fy, rx, ry, rp=None):
    dt = dtype_code(dt)
    check(L.lib.stk_residual(ctx.handle, dt, C.byref(grid), _ptr(vx, dt), _ptr(vy, dt), _ptr(p, dt), _ptr(eta_c, dt),
                             _ptr(eta_n, dt), _ptr(fx, dt), _ptr(fy, dt), _ptr(rx, dt), _ptr(ry, dt), _ptr(rp, dt)))


def energy_norm(ctx, dt, grid, vx, vy, p, eta_c, eta_n, fx, fy, allow_nonfinite=False):
    """(N_v, N_p, N_f, E, E_v) as a numpy array."""
    dt = dtype_code(dt)
    out = (C.c_double * 5)()
    rc = L.lib.stk_energy_norm(ctx.handle, dt, C.byref(grid), _ptr(vx, dt), _ptr(vy, dt), _ptr(p, dt),
                               _ptr(eta_c, dt), _ptr(eta_n, dt), _ptr(fx, dt), _ptr(fy, dt), out)
    if not (allow_nonfinite and rc == ENONFINITE):
        check(rc)
    return np.array(out[:])


def energy_norm_noalloc(ctx, dt, grid, vx, vy, p, eta_c, eta_n, fx, fy, out):
    """(N_v, N_p, N_f, E, E_v) into the device FP64 tensor ``out`` (>= 5
    elements), enqueued without waiting; the library allocates nothing."""
    dt = dtype_code(dt)
    if not (isinstance(out, torch.Tensor) and out.dtype == torch.float64 and out.numel() >= 5):
        raise ValueError("out must be a device float64 tensor of at least 5 elements")
    check(L.lib.stk_energy_norm_noalloc(ctx.handle, dt, C.byref(grid), _ptr(vx, dt), _ptr(vy, dt), _ptr(p, dt),
                                        _ptr(eta_c, dt), _ptr(eta_n, dt), _ptr(fx, dt), _ptr(fy, dt),
                                        _ptr(out, F64)))


def stream_probe(ctx, dt, grid, a, o):
    """The six-read, two-write streaming pass (a: 6 tensors, o: 2) over whole planes."""
    dt = dtype_code(dt)
    check(L.lib.stk_stream_probe(ctx.handle, dt, C.byref(grid), *[_ptr(t, dt) for t in a], *[_ptr(t, dt) for t in o]))


def ras_shifts(seed, n_outer, tile_x, tile_y):
    out = np.zeros(2 * n_outer, dtype=np.int32)
    check(L.lib.stk_ras_shifts(C.c_uint64(seed), int(n_outer), int(tile_x), int(tile_y),
                               out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out.reshape(n_outer, 2)


# ------------------------------------------------------------------ multigrid --

def mg_opts(nu1=2, nu2=2, omega=0.7, coarsest=8, fine_k=0, fine_halo=-1, coarse_smoother=0, coarse_tile=32,
            coarse_k=4, coarse_halo=0, sweep_growth=1.0, max_levels=0, stall_checks=0):
    """stk_mg_opts; coarse_smoother 'jacobi' / 'ras' (or 0 / 1)."""
    o = MgOpts()
    L.lib.stk_mg_opts_default(C.byref(o))
    o.nu1, o.nu2, o.omega, o.coarsest = int(nu1), int(nu2), float(omega), int(coarsest)
    o.fine_k, o.fine_halo = int(fine_k), int(fine_halo)
    o.coarse_smoother = {"jacobi": 0, "ras": 1}.get(coarse_smoother, coarse_smoother)
    o.coarse_tile, o.coarse_k, o.coarse_halo = int(coarse_tile), int(coarse_k), int(coarse_halo)
    o.sweep_growth, o.max_levels = float(sweep_growth), int(max_levels)
    o.stall_checks = int(stall_checks)
    return o


def _mode(mode):
    return MODES[mode] if isinstance(mode, str) else int(mode)


def _report(r):
    return dict(iterations=r.iterations, converged=bool(r.converged), ev=r.ev, nf=r.nf, seconds=r.seconds)


def mg_footprint(grid, mode="f64", **opts):
    n = C.c_size_t()
    check(L.lib.stk_mg_footprint(C.byref(grid), C.byref(mg_opts(**opts)), _mode(mode), C.byref(n)))
    return n.value


class MG:
    """stk_mg handle: hierarchy built from FP64 device viscosities (copied)."""

    def __init__(self, ctx, grid, eta_c, eta_n, **opts):
        self.ctx = ctx
        self.grid = grid
        self.handle = C.c_void_p()
        if not ctx.handle:
            raise ValueError("context is closed")
        check(L.lib.stk_mg_create(ctx.handle, C.byref(self.handle), C.byref(grid), _ptr(eta_c, F64),
                                  _ptr(eta_n, F64), C.byref(mg_opts(**opts))))
        ctx._mgs.add(self)

    def info(self):
        lv, cn, b = C.c_int(), C.c_int(), C.c_size_t()
        check(L.lib.stk_mg_info(self.handle, C.byref(lv), C.byref(cn), C.byref(b)))
        return dict(levels=lv.value, coarse_unknowns=cn.value, bytes=b.value)

    def bind(self, ctx, mode="f64"):
        """Move the handle to context ``ctx`` (same device), with the buffers of
        ``mode`` built first on the old context's stream."""
        check(L.lib.stk_mg_bind(self.handle, ctx.handle, _mode(mode)))
        self.ctx._mgs.discard(self)
        self.ctx = ctx
        ctx._mgs.add(self)

    def vcycle(self, dt, vx, vy, bx, by):
        dt = dtype_code(dt)
        check(L.lib.stk_mg_vcycle(self.handle, dt, _ptr(vx, dt), _ptr(vy, dt), _ptr(bx, dt), _ptr(by, dt)))

    def solve(self, mode, vx, vy, p, fx, fy, tol=1e-8, max_iters=500, allow_notconv=False):
        r = Report()
        rc = L.lib.stk_mg_solve(self.handle, _mode(mode), _ptr(vx, F64), _ptr(vy, F64), _ptr(p, F64),
                                _ptr(fx, F64), _ptr(fy, F64), float(tol), int(max_iters), C.byref(r))
        if not (allow_notconv and rc == ENOTCONV):
            check(rc)
        return _report(r)

    def close(self):
        if self.handle:
            check(L.lib.stk_mg_destroy(self.handle))  # EINVAL while the handle is in a batch
            self.handle = C.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def mg_solve_batch(ctx, mgs, mode, vx, vy, p, fx, fy, tol=1e-8, max_iters=500, allow_notconv=False):
    """Solve len(mgs) independent instances together (lists of device tensors)."""
    n = len(mgs)
    arr = lambda xs, dt=F64: (C.c_void_p * n)(*[_ptr(x, dt) for x in xs])
    hs = (C.c_void_p * n)(*[m.handle.value for m in mgs])
    reps = (Report * n)()
    pp = None if p is None else arr(p)
    rc = L.lib.stk_mg_solve_batch(ctx.handle, n, hs, _mode(mode), arr(vx), arr(vy), pp, arr(fx), arr(fy),
                                  float(tol), int(max_iters), reps)
    if not (allow_notconv and rc == ENOTCONV):
        check(rc)
    return [_report(r) for r in reps]


class Batch:
    """stk_batch: continuous batching of solves (instances join and leave between steps).

    ``add`` admits a solve and returns its slot; ``step`` advances every solve in
    flight by up to ``iters`` Krylov iterations and returns ``[(slot, report)]``
    for those that finished (their solutions are then in the arrays given to
    ``add``).  The tensors of a solve are kept alive here until it finishes."""

    def __init__(self, ctx, mode, max_slots):
        if not ctx.handle:
            raise ValueError("context is closed")
        self.ctx = ctx
        self.max_slots = int(max_slots)
        self.handle = C.c_void_p()
        check(L.lib.stk_batch_create(ctx.handle, _mode(mode), self.max_slots, C.byref(self.handle)))
        self._keep = {}
        self._done = (C.c_int * self.max_slots)()
        self._reps = (Report * self.max_slots)()
        ctx._batches.add(self)

    def add(self, mg, vx, vy, p, fx, fy, tol=1e-8, max_iters=500):
        slot = C.c_int()
        check(L.lib.stk_batch_add(self.handle, mg.handle, _ptr(vx, F64), _ptr(vy, F64), _ptr(p, F64),
                                  _ptr(fx, F64), _ptr(fy, F64), float(tol), int(max_iters), C.byref(slot)))
        self._keep[slot.value] = (mg, vx, vy, p, fx, fy)
        return slot.value

    def step(self, iters=1):
        nd = C.c_int()
        check(L.lib.stk_batch_step(self.handle, int(iters), self._done, self._reps, C.byref(nd)))
        out = []
        for k in range(nd.value):
            s = self._done[k]
            self._keep.pop(s, None)
            out.append((s, _report(self._reps[k])))
        return out

    def count(self):
        n = C.c_int()
        check(L.lib.stk_batch_count(self.handle, C.byref(n)))
        return n.value

    def close(self):
        if self.handle:
            L.lib.stk_batch_destroy(self.handle)
            self.handle = C.c_void_p()
            self._keep.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def uzawa_opts(omega_p=0.6, vcycles=1, tol=1e-8, max_cycles=1000, stages=0, stage_cycles=25, mode="f64"):
    o = L.UzawaOpts()
    L.lib.stk_uzawa_opts_default(C.byref(o))
    o.omega_p, o.vcycles, o.tol, o.max_cycles = float(omega_p), int(vcycles), float(tol), int(max_cycles)
    o.stages, o.stage_cycles, o.mode = int(stages), int(stage_cycles), _mode(mode)
    return o


def litho_pressure(ctx, grid, fy, p):
    """p <- lithostatic pressure of the vertical body force fy (zero mean)."""
    check(L.lib.stk_litho_pressure(ctx.handle, C.byref(grid), _ptr(fy, F64), _ptr(p, F64)))


def uzawa_pressure(ctx, grid, vx, vy, eta_c, omega_p, p):
    """p <- p + omega_p eta_c (-D v), then the mean removed (in place)."""
    check(L.lib.stk_uzawa_pressure(ctx.handle, C.byref(grid), _ptr(vx, F64), _ptr(vy, F64), _ptr(eta_c, F64),
                                   float(omega_p), _ptr(p, F64)))


def uzawa_solve(mg, grid, vx, vy, p, eta_c, eta_n, fx, fy, allow_notconv=False, **opts):
    """Inexact Uzawa cycles in place on (vx, vy, p); returns (report dict, E history)."""
    o = uzawa_opts(**opts)
    hist = (C.c_double * (o.max_cycles + 1))()
    r = L.UzawaReport()
    rc = L.lib.stk_uzawa_solve(mg.handle, C.byref(grid), _ptr(vx, F64), _ptr(vy, F64), _ptr(p, F64),
                               _ptr(eta_c, F64), _ptr(eta_n, F64), _ptr(fx, F64), _ptr(fy, F64), C.byref(o), hist,
                               C.byref(r))
    if not (allow_notconv and rc == ENOTCONV):
        check(rc)
    rep = dict(cycles=r.cycles, converged=bool(r.converged), e=r.e, ev=r.ev, seconds=r.seconds)
    return rep, np.array(hist[:r.cycles + 1])


def uzawa_anderson(mg, grid, vx, vy, p, eta_c, eta_n, fx, fy, depth=3, allow_notconv=False, **opts):
    """Anderson-accelerated Uzawa steps in place on (vx, vy, p); returns (report dict, E history)."""
    o = uzawa_opts(**opts)
    hist = (C.c_double * (o.max_cycles + 1))()
    r = L.UzawaReport()
    rc = L.lib.stk_uzawa_anderson(mg.handle, C.byref(grid), _ptr(vx, F64), _ptr(vy, F64), _ptr(p, F64),
                                  _ptr(eta_c, F64), _ptr(eta_n, F64), _ptr(fx, F64), _ptr(fy, F64), int(depth),
                                  C.byref(o), hist, C.byref(r))
    if not (allow_notconv and rc == ENOTCONV):
        check(rc)
    rep = dict(cycles=r.cycles, converged=bool(r.converged), e=r.e, ev=r.ev, seconds=r.seconds)
    return rep, np.array(hist[:r.cycles + 1])


# ------------------------------------------------------------------------ 3D --

def smooth3d_opts(omega=0.7, tile=8, halo=-1, k=2, shifts=None, seed=0):
    """Returns (Smooth3dOpts, keepalive); ``shifts`` is an (n_outer, 3) int array."""
    o = L.Smooth3dOpts()
    L.lib.stk_smooth3d_opts_default(C.byref(o))
    o.omega, o.tile, o.halo, o.k, o.seed = float(omega), int(tile), int(halo), int(k), C.c_uint64(seed).value
    keep = None
    if shifts is not None:
        keep = np.ascontiguousarray(np.asarray(shifts, dtype=np.int32).ravel())
        o.shifts = keep.ctypes.data_as(C.POINTER(C.c_int32))
    return o, keep


def _p3(ts, dt):
    return [_ptr(t, dt) for t in ts]


def smooth3d(ctx, dt, grid, v, eta, b, sweeps, variant="jacobi_fused", **opts):
    """In place on v = (vx, vy, vz); eta = (eta_c, eta_xy, eta_xz, eta_yz); b = (bx, by, bz)."""
    dt = dtype_code(dt)
    o, keep = smooth3d_opts(**opts)
    check(L.lib.stk_smooth3d(ctx.handle, dt, C.byref(grid), *_p3(v, dt), *_p3(eta, dt), *_p3(b, dt), int(sweeps),
                             VARIANTS[variant] if isinstance(variant, str) else int(variant), C.byref(o)))
    del keep


def ras_outer3d(ctx, dt, grid, v, eta, b, out, omega, tile, halo, kt, shift):
    dt = dtype_code(dt)
    check(L.lib.stk_ras_outer3d(ctx.handle, dt, C.byref(grid), *_p3(v, dt), *_p3(eta, dt), *_p3(b, dt),
                                *_p3(out, dt), float(omega), int(tile), int(halo), int(kt), *[int(s) for s in shift]))


def residual3d(ctx, dt, grid, v, eta, b, r):
    dt = dtype_code(dt)
    check(L.lib.stk_residual3d(ctx.handle, dt, C.byref(grid), *_p3(v, dt), *_p3(eta, dt), *_p3(b, dt), *_p3(r, dt)))


def energy_norm3d(ctx, dt, grid, v, eta, f):
    """(N_v, N_f, E_v) as a numpy array."""
    dt = dtype_code(dt)
    out = (C.c_double * 3)()
    check(L.lib.stk_energy_norm3d(ctx.handle, dt, C.byref(grid), *_p3(v, dt), *_p3(eta, dt), *_p3(f, dt), out))
    return np.array(out[:])

