"""ctypes wrappers over the FP64 C oracle (test infrastructure only).

Every function takes a *grid* object with attributes ``nx, ny, dx, dy,
eta_c, eta_n`` (numpy float64, natural shapes) and natural-shape numpy arrays;
see ``stokes_oracle.c`` for the layout and the operator definition (paper
Sec. 2.1 equations, Fig. 1 staggering).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        I = C.c_int
        D = C.c_double
        sig = {
            "or_apply": [I, I, D, D, P, P, P, P, P, P],
            "or_diag": [I, I, D, D, P, P, P, P],
            "or_rhs": [I, I, D, D, P, P, P, P, P],
            "or_divergence": [I, I, D, D, P, P, P],
            "or_jacobi": [I, I, D, D, P, P, P, P, D, P, P, P, P],
            "or_rbgs": [I, I, D, D, P, P, P, P, D, P, P],
            "or_ras": [I, I, D, D, P, P, P, P, D, I, I, I, I, I, I, P, P, P, P],
            "or_energy": [I, I, D, D, P, P, P, P, P, P, P, P],
            "or_prolong_add": [I, I, P, P, P, P],
            "or_restrict": [I, I, P, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = I
        L.or_set_num_threads.argtypes = [I]
        L.or_set_num_threads.restype = None
        _lib = L
    return _lib


def num_threads():
    return int(lib().or_num_threads())


def set_num_threads(n):
    """Threads of the following oracle calls (OpenMP)."""
    lib().or_set_num_threads(int(n))


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, "oracle wants C-contiguous float64"
    return a.ctypes.data


def _f(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == shape, (a.shape, shape)
    return a


def _shapes(g):
    return (g.ny, g.nx + 1), (g.ny + 1, g.nx)


def _ge(g):
    return (g.nx, g.ny, float(g.dx), float(g.dy), _p(_f(g.eta_c, (g.ny, g.nx))),
            _p(_f(g.eta_n, (g.ny + 1, g.nx + 1))))


def apply(g, vx, vy):
    """(M v)_x, (M v)_y on the unknowns (0 on walls)."""
    sx, sy = _shapes(g)
    vx, vy = _f(vx, sx), _f(vy, sy)
    mx, my = np.empty(sx), np.empty(sy)
    ec, en = _f(g.eta_c, (g.ny, g.nx)), _f(g.eta_n, (g.ny + 1, g.nx + 1))
    lib().or_apply(g.nx, g.ny, g.dx, g.dy, _p(ec), _p(en), _p(vx), _p(vy), _p(mx), _p(my))
    return mx, my


def diag(g):
    """d = diag(-M) on the unknowns (0 on walls)."""
    sx, sy = _shapes(g)
    dx_, dy_ = np.empty(sx), np.empty(sy)
    ec, en = _f(g.eta_c, (g.ny, g.nx)), _f(g.eta_n, (g.ny + 1, g.nx + 1))
    lib().or_diag(g.nx, g.ny, g.dx, g.dy, _p(ec), _p(en), _p(dx_), _p(dy_))
    return dx_, dy_


def rhs(g, fx, fy, p=None):
    """b = f - G p on the unknowns (0 on walls)."""
    sx, sy = _shapes(g)
    fx, fy = _f(fx, sx), _f(fy, sy)
    pp = None if p is None else _f(p, (g.ny, g.nx))
    bx, by = np.empty(sx), np.empty(sy)
    lib().or_rhs(g.nx, g.ny, g.dx, g.dy, _p(fx), _p(fy), _p(pp), _p(bx), _p(by))
    return bx, by


def divergence(g, vx, vy):
    sx, sy = _shapes(g)
    vx, vy = _f(vx, sx), _f(vy, sy)
    dv = np.empty((g.ny, g.nx))
    lib().or_divergence(g.nx, g.ny, g.dx, g.dy, _p(vx), _p(vy), _p(dv))
    return dv


def residual(g, vx, vy, fx, fy, p=None):
    """r_v = b - M v (0 on walls) and r_p = -D v."""
    bx, by = rhs(g, fx, fy, p)
    mx, my = apply(g, vx, vy)
    return bx - mx, by - my, -divergence(g, vx, vy)


def jacobi(g, bx, by, omega, vx, vy):
    """One damped Jacobi sweep, returns the new (vx, vy)."""
    sx, sy = _shapes(g)
    vx, vy, bx, by = _f(vx, sx), _f(vy, sy), _f(bx, sx), _f(by, sy)
    ox, oy = np.empty(sx), np.empty(sy)
    ec, en = _f(g.eta_c, (g.ny, g.nx)), _f(g.eta_n, (g.ny + 1, g.nx + 1))
    lib().or_jacobi(g.nx, g.ny, g.dx, g.dy, _p(ec), _p(en), _p(bx), _p(by), float(omega),
                    _p(vx), _p(vy), _p(ox), _p(oy))
    return ox, oy


def rbgs(g, bx, by, omega, vx, vy):
    """One red-black Gauss-Seidel sweep (vx-red, vx-black, vy-red, vy-black)."""
    sx, sy = _shapes(g)
    ox, oy = np.array(_f(vx, sx)), np.array(_f(vy, sy))
    bx, by = _f(bx, sx), _f(by, sy)
    ec, en = _f(g.eta_c, (g.ny, g.nx)), _f(g.eta_n, (g.ny + 1, g.nx + 1))
    lib().or_rbgs(g.nx, g.ny, g.dx, g.dy, _p(ec), _p(en), _p(bx), _p(by), float(omega), _p(ox), _p(oy))
    return ox, oy


def ras_outer(g, bx, by, omega, tile_x, tile_y, halo, kt, sx_, sy_, vx, vy):
    """One RAS outer iteration (Alg. 2, snapshot semantics) with shift (sx_, sy_)."""
    sx, sy = _shapes(g)
    vx, vy, bx, by = _f(vx, sx), _f(vy, sy), _f(bx, sx), _f(by, sy)
    ox, oy = np.empty(sx), np.empty(sy)
    ec, en = _f(g.eta_c, (g.ny, g.nx)), _f(g.eta_n, (g.ny + 1, g.nx + 1))
    lib().or_ras(g.nx, g.ny, g.dx, g.dy, _p(ec), _p(en), _p(bx), _p(by), float(omega),
                 int(tile_x), int(tile_y), int(halo), int(kt), int(sx_), int(sy_),
                 _p(vx), _p(vy), _p(ox), _p(oy))
    return ox, oy


def energy(g, vx, vy, fx, fy, p=None):
    """(N_v, N_p, N_f, E, E_v) of Sec. 6.4 (see stokes_oracle.c)."""
    sx, sy = _shapes(g)
    vx, vy, fx, fy = _f(vx, sx), _f(vy, sy), _f(fx, sx), _f(fy, sy)
    pp = None if p is None else _f(p, (g.ny, g.nx))
    out = np.empty(5)
    ec, en = _f(g.eta_c, (g.ny, g.nx)), _f(g.eta_n, (g.ny + 1, g.nx + 1))
    lib().or_energy(g.nx, g.ny, g.dx, g.dy, _p(ec), _p(en), _p(fx), _p(fy), _p(pp), _p(vx), _p(vy), _p(out))
    return out


# ---------------------------------------------------------------- smoothers --

def n_outer(sweeps, k, last_partial=True):
    """Outer RAS iterations and the sweep count of each (Alg. 2: ceil(N/k);
    with ``last_partial`` the last one runs only the remainder)."""
    if sweeps <= 0:
        return []
    n = -(-sweeps // k)
    ks = [k] * n
    if last_partial and sweeps % k:
        ks[-1] = sweeps % k
    return ks


def smooth(g, vx, vy, fx, fy, p, sweeps, variant, omega=None, tile_x=64, tile_y=64, halo=None,
           k=4, shifts=None, last_partial=True):
    """Reference for the library's smooth call: ``sweeps`` sweeps of
    ``variant`` in {"jacobi", "jacobi_fused", "ras", "rbgs"} on M v = f - G p."""
    bx, by = rhs(g, fx, fy, p)
    if omega is None:
        omega = 1.0 if variant == "rbgs" else 0.7
    vx, vy = np.array(vx, dtype=np.float64), np.array(vy, dtype=np.float64)
    if variant in ("jacobi", "jacobi_fused"):
        for _ in range(sweeps):
            vx, vy = jacobi(g, bx, by, omega, vx, vy)
    elif variant == "rbgs":
        for _ in range(sweeps):
            vx, vy = rbgs(g, bx, by, omega, vx, vy)
    elif variant == "ras":
        h = k if halo is None else halo
        ks = n_outer(sweeps, k, last_partial)
        assert shifts is not None and len(shifts) >= len(ks)
        for t, kt in enumerate(ks):
            vx, vy = ras_outer(g, bx, by, omega, tile_x, tile_y, h, kt, shifts[t][0], shifts[t][1], vx, vy)
    else:
        raise ValueError(variant)
    # walls are Dirichlet 0 on output
    vx[:, 0] = vx[:, -1] = 0.0
    vy[0, :] = vy[-1, :] = 0.0
    return vx, vy


# ---------------------------------------------------------------- transfers --

def prolong_add(nx, ny, cx, cy, fx, fy):
    NX, NY = nx // 2, ny // 2
    cx, cy = _f(cx, (NY, NX + 1)), _f(cy, (NY + 1, NX))
    fx, fy = np.array(_f(fx, (ny, nx + 1))), np.array(_f(fy, (ny + 1, nx)))
    lib().or_prolong_add(nx, ny, _p(cx), _p(cy), _p(fx), _p(fy))
    return fx, fy


def restrict(nx, ny, fx, fy):
    NX, NY = nx // 2, ny // 2
    fx, fy = _f(fx, (ny, nx + 1)), _f(fy, (ny + 1, nx))
    cx, cy = np.empty((NY, NX + 1)), np.empty((NY + 1, NX))
    lib().or_restrict(nx, ny, _p(fx), _p(fy), _p(cx), _p(cy))
    return cx, cy
