"""Seeded synthetic inputs for the staggered-grid Stokes velocity smoother.

This module only *builds input fields*; it holds none of the smoother's,
residual's or multigrid's arithmetic.  Both the CPU oracle (tests) and the
HIP path (tests, bench) are fed from here.

Grid convention (paper Sec. 2.1, staggered grid of Fig. 1; unit square, y up):
  * cell (i, j), 0 <= i < nx, 0 <= j < ny, centre ((i+1/2)dx, (j+1/2)dy):
    carries the cell viscosity eta_c (the paper's eta_P) and the pressure p;
  * node (i, j), 0 <= i <= nx, 0 <= j <= ny, at (i dx, j dy): eta_n (eta_B);
  * vx(i, j) at (i dx, (j+1/2)dy): array shape (ny, nx+1);
  * vy(i, j) at ((i+1/2)dx, j dy): array shape (ny+1, nx);
  * density rho lives with vy (Fig. 1 caption), so fy has the vy shape.

Problem family: the sinker benchmark of Sec. 6.1 (stiff, dense circular
inclusions in a weaker medium, gravity pointing down), made non-dimensional.
Right-hand side: with y up and gravity (0, -|g|), the momentum balance
div(sigma') - grad p + rho g = 0 gives f = -rho g, i.e. fx = 0, fy = +rho|g|.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    nx: int
    ny: int
    dx: float
    dy: float
    eta_c: np.ndarray          # (ny, nx)
    eta_n: np.ndarray          # (ny+1, nx+1)
    fx: np.ndarray             # (ny, nx+1)
    fy: np.ndarray             # (ny+1, nx)
    meta: dict = field(default_factory=dict)

    def zeros_v(self):
        return (np.zeros((self.ny, self.nx + 1)), np.zeros((self.ny + 1, self.nx)))


def _inside(x, y, sinkers):
    """Mask (len(y), len(x)) of the points (x[i], y[j]) inside any circle,
    evaluated on each circle's bounding box only."""
    m = np.zeros((len(y), len(x)), dtype=bool)
    for (cx, cy, r) in sinkers:
        i0, i1 = np.searchsorted(x, cx - r, "left"), np.searchsorted(x, cx + r, "right")
        j0, j1 = np.searchsorted(y, cy - r, "left"), np.searchsorted(y, cy + r, "right")
        if i0 >= i1 or j0 >= j1:
            continue
        m[j0:j1, i0:i1] |= (x[None, i0:i1] - cx) ** 2 + (y[j0:j1, None] - cy) ** 2 <= r * r
    return m


def nodal_harmonic(eta_c: np.ndarray) -> np.ndarray:
    """Nodal viscosity: harmonic mean of the 1, 2 or 4 cells touching a node.

    Input construction only (how eta_B is obtained from eta_P is not fixed by
    the paper; the harmonic rule is the workload's stated choice)."""
    ny, nx = eta_c.shape
    inv = 1.0 / eta_c
    s = np.zeros((ny + 1, nx + 1))
    n = np.zeros((ny + 1, nx + 1))
    for oj in (0, 1):
        for oi in (0, 1):
            s[oj:oj + ny, oi:oi + nx] += inv
            n[oj:oj + ny, oi:oi + nx] += 1.0
    return n / s


def sinker_problem(nx: int, ny: int, sinkers, eta_in: float, eta_out,
                   rho_in: float = 1.1, rho_out: float = 1.0, g: float = 1.0,
                   meta: dict | None = None) -> Problem:
    """Fields for circular inclusions ``sinkers = [(cx, cy, r), ...]``.

    ``eta_out`` is a scalar or a (ny, nx) background array."""
    dx, dy = 1.0 / nx, 1.0 / ny
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    ins = _inside(xc, yc, sinkers)
    bg = np.broadcast_to(np.asarray(eta_out, dtype=np.float64), (ny, nx))
    eta_c = np.where(ins, eta_in, bg).astype(np.float64)
    eta_n = nodal_harmonic(eta_c)
    # density sampled at the vy points ((i+1/2)dx, j dy)
    rho = np.where(_inside(xc, np.arange(ny + 1) * dy, sinkers), rho_in, rho_out)
    fy = (rho * g).astype(np.float64)
    fx = np.zeros((ny, nx + 1))
    return Problem(nx, ny, dx, dy, eta_c, eta_n, fx, fy, dict(meta or {}))


# --------------------------------------------------------------------------
# The workloads (non-dimensional sinker family, Sec. 6.1 / Sec. 7.1 shapes)
# --------------------------------------------------------------------------

def centred_sinker(n: int = 64) -> Problem:
    """One centred sinker, r = 0.1, eta 1e3 inside / 1 outside, rho 1.1 / 1.0."""
    return sinker_problem(n, n, [(0.5, 0.5, 0.1)], 1e3, 1.0,
                          meta=dict(workload="centred_sinker", n=n))


def random_sinkers(n: int, count: int, seed: int, eta_in: float = 1e6,
                   eta_out=1.0, rmin: float = 0.02, rmax: float = 0.08) -> Problem:
    """``count`` sinkers, centres U[0.1,0.9]^2, radii U[rmin, rmax]."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 0.9, size=(count, 2))
    r = rng.uniform(rmin, rmax, size=count)
    sinkers = [(float(c[k, 0]), float(c[k, 1]), float(r[k])) for k in range(count)]
    return sinker_problem(n, n, sinkers, eta_in, eta_out,
                          meta=dict(workload="random_sinkers", n=n, count=count, seed=seed))


def smoother_workload(n: int = 4096, seed: int = 2) -> Problem:
    """8 seeded sinkers, eta 1e6 / 1, harmonic nodal eta (smoother throughput)."""
    return random_sinkers(n, 8, seed)


def smooth_log_uniform_field(n: int, seed: int, lo: float = -2.0, hi: float = 4.0, kmax: int = 8,
                             modes: int = 64) -> np.ndarray:
    """(n, n) cell field with log10 values spread uniformly over [lo, hi] and
    spatially smooth: a Gaussian random field of unit variance (``modes`` plane
    waves, integer wavenumbers |k| <= kmax, random phases; correlation length
    ~ 1/kmax of the domain) mapped through the normal CDF to U(0, 1), then to
    [lo, hi].  Written as one rank-2*modes product so that 8192^2 takes seconds."""
    from scipy.special import ndtr
    rng = np.random.default_rng(seed)
    k = rng.integers(-kmax, kmax + 1, size=(modes, 2))
    k[(k == 0).all(axis=1)] = (1, 0)
    ph = rng.uniform(0.0, 2.0 * np.pi, modes)
    x = (np.arange(n) + 0.5) / n
    a = 2.0 * np.pi * np.outer(x, k[:, 0])            # (n, modes): x phase
    b = 2.0 * np.pi * np.outer(x, k[:, 1]) + ph       # (n, modes): y phase
    # cos(a + b) = cos b cos a - sin b sin a, summed over modes: rows y, columns x
    U = np.concatenate([np.cos(b), -np.sin(b)], axis=1)
    V = np.concatenate([np.cos(a), np.sin(a)], axis=1)
    g = (U @ V.T) * np.sqrt(2.0 / modes)
    return 10.0 ** (lo + (hi - lo) * ndtr(g))


def lognormal_background_workload(n: int = 8192, seed: int = 4, count: int = 16) -> Problem:
    """16 sinkers of eta 1e6 over a smooth background whose log10(eta) is
    uniform on [-2, 4] (``smooth_log_uniform_field``): the multigrid /
    refinement workload, viscosity contrast up to 1e8."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 0.9, size=(count, 2))
    r = rng.uniform(0.02, 0.08, size=count)
    bg = smooth_log_uniform_field(n, seed)
    sinkers = [(float(c[k, 0]), float(c[k, 1]), float(r[k])) for k in range(count)]
    return sinker_problem(n, n, sinkers, 1e6, bg,
                          meta=dict(workload="log_uniform_background", n=n, count=count, seed=seed))


def iid_log_uniform_workload(n: int = 8192, seed: int = 4, count: int = 16) -> Problem:
    """The refinement workload with the literal background: log10(eta) drawn
    i.i.d. per cell from U(-2, 4) (up to six decades between neighbouring
    cells), the same 16 sinkers of eta 1e6."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 0.9, size=(count, 2))
    r = rng.uniform(0.02, 0.08, size=count)
    bg = 10.0 ** np.random.default_rng(seed + 1).uniform(-2.0, 4.0, size=(n, n))
    sinkers = [(float(c[k, 0]), float(c[k, 1]), float(r[k])) for k in range(count)]
    return sinker_problem(n, n, sinkers, 1e6, bg,
                          meta=dict(workload="iid_log_uniform_background", n=n, count=count, seed=seed))


def instance_problem(n: int, rng: np.random.Generator) -> Problem:
    """One request/instance: sinker count U{1..8}, contrast 10^U(2,6)."""
    count = int(rng.integers(1, 9))
    contrast = float(10.0 ** rng.uniform(2.0, 6.0))
    c = rng.uniform(0.1, 0.9, size=(count, 2))
    r = rng.uniform(0.02, 0.08, size=count)
    sinkers = [(float(c[k, 0]), float(c[k, 1]), float(r[k])) for k in range(count)]
    return sinker_problem(n, n, sinkers, contrast, 1.0,
                          meta=dict(workload="instance", n=n, count=count, contrast=contrast))


def batch_mix(seed: int = 5, sizes=((256, 28), (512, 20), (1024, 12), (2048, 4))):
    """Uneven mix of independent sinker problems (default: 64 instances)."""
    rng = np.random.default_rng(seed)
    out = []
    for n, cnt in sizes:
        for _ in range(cnt):
            out.append(instance_problem(n, rng))
    order = rng.permutation(len(out))
    return [out[k] for k in order]


def random_velocity(p: Problem, seed: int, scale: float = 1.0):
    """Random velocity state with Dirichlet wall entries set to 0."""
    rng = np.random.default_rng(seed)
    vx = rng.standard_normal((p.ny, p.nx + 1)) * scale
    vy = rng.standard_normal((p.ny + 1, p.nx)) * scale
    vx[:, 0] = 0.0
    vx[:, -1] = 0.0
    vy[0, :] = 0.0
    vy[-1, :] = 0.0
    return vx, vy


def random_pressure(p: Problem, seed: int, scale: float = 1.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((p.ny, p.nx)) * scale


def random_shifts(n_outer: int, tile_x: int, tile_y: int, seed: int) -> np.ndarray:
    """Explicit tile shifts (sx, sy) per outer iteration, int32 (n_outer, 2)."""
    rng = np.random.default_rng(seed)
    s = np.empty((n_outer, 2), dtype=np.int32)
    s[:, 0] = rng.integers(0, tile_x, size=n_outer)
    s[:, 1] = rng.integers(0, tile_y, size=n_outer)
    return s


# --------------------------------------------------------------------------
# 3D problems (the paper's future-work extension): spherical sinkers in a
# free-slip unit box, gravity along -z
# --------------------------------------------------------------------------

@dataclass
class Problem3:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    eta_c: np.ndarray   # (nz, ny, nx) cells
    eta_xy: np.ndarray  # (nz, ny+1, nx+1) z-parallel edges
    eta_xz: np.ndarray  # (nz+1, ny, nx+1) y-parallel edges
    eta_yz: np.ndarray  # (nz+1, ny+1, nx) x-parallel edges
    fx: np.ndarray = None  # (nz, ny, nx+1)
    fy: np.ndarray = None  # (nz, ny+1, nx)
    fz: np.ndarray = None  # (nz+1, ny, nx)
    meta: dict = field(default_factory=dict)

    def zeros_v(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return np.zeros((nz, ny, nx + 1)), np.zeros((nz, ny + 1, nx)), np.zeros((nz + 1, ny, nx))


def edge_harmonic(eta_c: np.ndarray, axis: int) -> np.ndarray:
    """Viscosity on the edges that run along array axis `axis` of the (z, y, x)
    cell array (0: z-parallel, 1: y-parallel, 2: x-parallel edges): harmonic
    mean of the 1, 2 or 4 cells that touch the edge.  Input construction only
    (the workload's stated choice, as for the 2D nodes)."""
    nz, ny, nx = eta_c.shape
    inv = 1.0 / eta_c
    # an edge parallel to `axis` sits between cells along the two other axes
    shape = [nz + (axis != 0), ny + (axis != 1), nx + (axis != 2)]
    s = np.zeros(shape)
    n = np.zeros(shape)
    others = [a for a in range(3) if a != axis]
    for o0 in (0, 1):
        for o1 in (0, 1):
            sl = [slice(None)] * 3
            for a, o in zip(others, (o0, o1)):
                size = eta_c.shape[a]
                sl[a] = slice(o, o + size)
            s[tuple(sl)] += inv
            n[tuple(sl)] += 1.0
    return n / s


def sinker_problem3d(nx: int, ny: int, nz: int, spheres, eta_in: float, eta_out: float, rho_in: float = 1.1,
                     rho_out: float = 1.0, g: float = 1.0, meta: dict | None = None) -> Problem3:
    """Spheres ``[(cx, cy, cz, r), ...]`` of viscosity eta_in and density rho_in
    in a medium of eta_out, rho_out; fz = rho g at the vz faces (gravity -z)."""
    dx, dy, dz = 1.0 / nx, 1.0 / ny, 1.0 / nz
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    zc = (np.arange(nz) + 0.5) * dz

    def inside(x, y, z):
        m = np.zeros((len(z), len(y), len(x)), bool)
        for (cx, cy, cz, r) in spheres:
            m |= ((x[None, None, :] - cx) ** 2 + (y[None, :, None] - cy) ** 2 + (z[:, None, None] - cz) ** 2) <= r * r
        return m

    eta_c = np.where(inside(xc, yc, zc), eta_in, eta_out).astype(np.float64)
    rho = np.where(inside(xc, yc, np.arange(nz + 1) * dz), rho_in, rho_out)
    return Problem3(nx, ny, nz, dx, dy, dz, eta_c, edge_harmonic(eta_c, 0), edge_harmonic(eta_c, 1),
                    edge_harmonic(eta_c, 2), np.zeros((nz, ny, nx + 1)), np.zeros((nz, ny + 1, nx)),
                    (rho * g).astype(np.float64), dict(meta or {}))


def random_sinkers3d(n: int, count: int, seed: int, eta_in: float = 1e4, eta_out: float = 1.0,
                     rmin: float = 0.05, rmax: float = 0.15) -> Problem3:
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.15, 0.85, size=(count, 3))
    r = rng.uniform(rmin, rmax, size=count)
    return sinker_problem3d(n, n, n, [(*map(float, c[q]), float(r[q])) for q in range(count)], eta_in, eta_out,
                            meta=dict(workload="random_sinkers3d", n=n, count=count, seed=seed))


def random_velocity3d(p: Problem3, seed: int, scale: float = 1.0):
    """Random velocity state with the wall entries set to 0."""
    rng = np.random.default_rng(seed)
    vx, vy, vz = (rng.standard_normal(a.shape) * scale for a in p.zeros_v())
    vx[:, :, 0] = vx[:, :, -1] = 0.0
    vy[:, 0, :] = vy[:, -1, :] = 0.0
    vz[0, :, :] = vz[-1, :, :] = 0.0
    return vx, vy, vz
