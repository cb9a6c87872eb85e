"""Python face of the stk C ABI (same call names, torch tensors for memory).

Arguments are device tensors (or raw device pointers as ints); this module
only checks and marshals them.  See ``include/stk.h`` for the semantics.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import (EHIP, EINVAL, ENOMEM, ENONFINITE, ENOTCONV, EUNSUPPORTED, F32, F64, JACOBI, JACOBI_FUSED, OK,
                   RAS_JACOBI, RBGS, VARIANTS, Grid, SmoothOpts, StkError, check)

__all__ = ["Context", "Grid", "SmoothOpts", "StkError", "smooth", "ras_outer", "residual", "energy_norm", "ras_shifts",
           "smooth_opts", "F64", "F32", "JACOBI", "JACOBI_FUSED", "RAS_JACOBI", "RBGS", "VARIANTS", "OK", "EINVAL",
           "ENOMEM", "EHIP", "ENOTCONV", "ENONFINITE", "EUNSUPPORTED", "dtype_code", "torch_dtype"]


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


class Context:
    """stk_ctx bound to a device and a HIP stream (default: torch's current)."""

    def __init__(self, device: int = 0, stream=None):
        self.device = device
        self.handle = C.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream(device)
        sp = s.cuda_stream if hasattr(s, "cuda_stream") else s
        check(L.lib.stk_ctx_create(C.byref(self.handle), device, C.c_void_p(sp)))

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
        if self.handle:
            L.lib.stk_ctx_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
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


def ras_shifts(seed, n_outer, tile_x, tile_y):
    out = np.zeros(2 * n_outer, dtype=np.int32)
    check(L.lib.stk_ras_shifts(C.c_uint64(seed), int(n_outer), int(tile_x), int(tile_y),
                               out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out.reshape(n_outer, 2)
