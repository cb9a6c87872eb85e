"""FP64 geometric multigrid V-cycle and Krylov solve (test infrastructure).

The paper solves the velocity block M v = f - G p with a matrix-free
geometric multigrid whose smoothing dominates the cost (Sec. 3.2, Sec. 6.2);
it does not print the transfer operators, the coarse operators or the
coarsest-grid solver.  This oracle takes the following reading:

  * coarsening by 2 in x and y while min(nx, ny) > coarsest and both even;
  * bilinear prolongation P and restriction R = P^T / 4 (``oracle.sparse``);
  * Galerkin coarse operators M_c = R M P (= P^T M P / 4).  Rediscretised
    coarse operators (coarse viscosities by averaging) were tried first and
    lose convergence at viscosity contrasts >= ~1e3-1e6 even inside a Krylov
    method; with Galerkin operators the coarse correction is an A-orthogonal
    projection and the contrast-1e6 solves converge;
  * smoother S = damped Jacobi (RAS blocking with halo >= k-1 produces exactly
    Jacobi^k, Alg. 2 with enough overlap);
  * coarsest grid: exact FP64 solve (Cholesky of -M_c);
  * V(nu1, nu2): pre-smooth, residual, restrict, recurse from 0, prolong-add,
    post-smooth;
  * solve: V-cycle-preconditioned flexible conjugate gradients on the SPD
    system -M v = -b, stopping on the velocity energy residual
    E_v = sqrt(N_v/N_f) <= tol (Sec. 6.4).  The paper's own accelerator is
    Anderson acceleration (Sec. 3.3 / Alg. 1), of the same Krylov family.

Internally level l works on packed unknown vectors with A_l = -M_l (SPD).
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np
import scipy.linalg as sla

from . import sparse as SP
from . import stokes as S


def hierarchy(g, coarsest=8):
    L0 = SimpleNamespace(nx=g.nx, ny=g.ny, dx=g.dx, dy=g.dy, eta_c=np.asarray(g.eta_c, float),
                         eta_n=np.asarray(g.eta_n, float))
    L0.A = SP.operator_matrix(L0)
    levels = [L0]
    while True:
        L = levels[-1]
        if min(L.nx, L.ny) <= coarsest or L.nx % 2 or L.ny % 2:
            break
        L.P = SP.prolongation_matrix(L.nx, L.ny)
        C = SimpleNamespace(nx=L.nx // 2, ny=L.ny // 2, dx=2 * L.dx, dy=2 * L.dy)
        C.A = (0.25 * (L.P.T @ L.A @ L.P)).tocsr()
        levels.append(C)
    for L in levels:
        L.D = L.A.diagonal()
    C = levels[-1]
    C.chol = sla.cho_factor(C.A.toarray())
    return levels


def _vcycle_packed(levels, l, x, c, nu1, nu2, omega):
    """One V-cycle for A_l x = c from x."""
    L = levels[l]
    if l == len(levels) - 1:
        return sla.cho_solve(L.chol, c)
    for _ in range(nu1):
        x = x + omega * (c - L.A @ x) / L.D
    cc = 0.25 * (L.P.T @ (c - L.A @ x))
    xc = _vcycle_packed(levels, l + 1, np.zeros(len(cc)), cc, nu1, nu2, omega)
    x = x + L.P @ xc
    for _ in range(nu2):
        x = x + omega * (c - L.A @ x) / L.D
    return x


def vcycle(levels, l, vx, vy, bx, by, nu1=2, nu2=2, omega=0.7):
    """One V-cycle for M v = b on level l (natural arrays, walls 0)."""
    L = levels[l]
    x = SP.pack(L.nx, L.ny, vx, vy)
    c = -SP.pack(L.nx, L.ny, bx, by)  # A x = -b
    return SP.unpack(L.nx, L.ny, _vcycle_packed(levels, l, x, c, nu1, nu2, omega))


_vcycle_natural = vcycle


def coarse_solve(L, bx, by):
    """Exact solution of M v = b on the coarsest level."""
    return SP.unpack(L.nx, L.ny, sla.cho_solve(L.chol, -SP.pack(L.nx, L.ny, bx, by)))


# ---------------------------------------------------------------------------
# Smoother variants inside the V-cycle (Sec. 6.2, 6.3): RAS-type temporal
# blocking (Alg. 2) on a level's assembled operator, the mixed smoother
# (Jacobi on the finest level, RAS on the coarser ones), sweep counts growing
# per level, and a truncated hierarchy whose coarsest level is relaxed.
# ---------------------------------------------------------------------------

def tile_intervals(n, T, s):
    """Tiles along one axis: intervals between the cuts {s + mT} inside (0, n),
    clipped to [0, n) (Alg. 2's shifted tiling; edge tiles may be partial)."""
    cuts = [c for c in range(s % T, n, T) if c > 0]
    edges = [0] + cuts + [n]
    return [(edges[q], edges[q + 1]) for q in range(len(edges) - 1)]


def _cell_unknowns(vx_id, vy_id, x0, x1, y0, y1):
    """Packed unknowns associated with the cells [x0, x1) x [y0, y1): the
    left-face vx(i, j) and the bottom-face vy(i, j) of each cell."""
    e = np.concatenate([vx_id[y0:y1, x0:x1].ravel(), vy_id[y0:y1, x0:x1].ravel()])
    return e[e >= 0]


def ras_level(L, x, c, T, h, k, omega, shift=(0, 0)):
    """One RAS outer iteration (Alg. 2 with snapshot semantics) for A_l x = c
    on level L: every tile's owned cells grown by h (clipped) form the region
    E; k damped-Jacobi sweeps update the unknowns of E while every unknown
    outside E keeps its snapshot value; the unknowns of the owned cells are
    written back.  Tiles are T x T cells, cut at the given shift."""
    _, vx_id, vy_id = SP.numbering(L.nx, L.ny)
    u = np.array(x, dtype=float)
    out = u.copy()
    for (x0, x1) in tile_intervals(L.nx, T, shift[0]):
        for (y0, y1) in tile_intervals(L.ny, T, shift[1]):
            E = _cell_unknowns(vx_id, vy_id, max(x0 - h, 0), min(x1 + h, L.nx), max(y0 - h, 0), min(y1 + h, L.ny))
            own = _cell_unknowns(vx_id, vy_id, x0, x1, y0, y1)
            AE = L.A[E]
            z = u.copy()
            for _ in range(k):
                z[E] = z[E] + omega * (c[E] - AE @ z) / L.D[E]
            out[own] = z[own]
    return out


def sweeps_per_level(nu, growth, l):
    """nu * growth^l rounded to the nearest integer (halves up)."""
    return int(np.floor(nu * growth ** l + 0.5))


def _smooth_level(L, l, x, c, nu, omega, fine, coarse):
    """nu sweeps of level l's smoother: Jacobi, or RAS outer iterations of
    k_t = min(k, sweeps left) sweeps each (tile T, halo h, shift 0) when a RAS
    setting is given for this level (`fine` for l = 0, `coarse` for l >= 1)."""
    ras = fine if l == 0 else coarse
    if not ras:
        for _ in range(nu):
            x = x + omega * (c - L.A @ x) / L.D
        return x
    left = nu
    while left > 0:
        kt = min(ras["k"], left)
        x = ras_level(L, x, c, ras["T"], ras["h"], kt, omega)
        left -= kt
    return x


def hierarchy_truncated(g, max_levels, coarsest=8):
    """The Galerkin hierarchy of ``hierarchy`` cut after ``max_levels`` levels
    (0: no cut)."""
    levels = hierarchy(g, coarsest=coarsest)
    if max_levels and len(levels) > max_levels:
        levels = levels[:max_levels]
        C = levels[-1]
        del C.P
        n = C.A.shape[0]
        C.chol = sla.cho_factor(C.A.toarray()) if n <= 4096 else None
    return levels


def vcycle_general(levels, l, x, c, nu1=2, nu2=2, omega=0.7, growth=1.0, fine=None, coarse=None,
                   relax_coarsest=False):
    """One V-cycle for A_l x = c (packed unknowns) with the smoother variants:
    level l takes nu1 * growth^l pre- and nu2 * growth^l post-sweeps of its
    smoother (``_smooth_level``); the coarsest level is solved exactly, or,
    with ``relax_coarsest``, relaxed by its pre- and post-sweeps from x."""
    L = levels[l]
    n1, n2 = sweeps_per_level(nu1, growth, l), sweeps_per_level(nu2, growth, l)
    if l == len(levels) - 1:
        if relax_coarsest:
            return _smooth_level(L, l, x, c, n1 + n2, omega, fine, coarse)
        return sla.cho_solve(L.chol, c)
    x = _smooth_level(L, l, x, c, n1, omega, fine, coarse)
    cc = 0.25 * (L.P.T @ (c - L.A @ x))
    xc = vcycle_general(levels, l + 1, np.zeros(len(cc)), cc, nu1, nu2, omega, growth, fine, coarse, relax_coarsest)
    x = x + L.P @ xc
    return _smooth_level(L, l, x, c, n2, omega, fine, coarse)


def _dot(a, b):
    return float(np.sum(a[0] * b[0]) + np.sum(a[1] * b[1]))


def _masked_energy(rx, ry, dxg, dyg):
    mx, my = dxg > 0, dyg > 0
    return float(np.sum(np.where(mx, rx * rx / np.where(mx, dxg, 1.0), 0.0)) +
                 np.sum(np.where(my, ry * ry / np.where(my, dyg, 1.0), 0.0)))


def pcg(levels, fx, fy, p=None, tol=1e-8, max_iters=500, nu1=2, nu2=2, omega=0.7, x0=None, variants=None):
    """Flexible conjugate gradients on A x = -b (A = -M SPD, b = f - G p),
    preconditioned by one V-cycle per iteration, in FP64.  Stops when the
    velocity energy residual E_v = sqrt(N_v / N_f) of Sec. 6.4 is <= tol.
    When the recurrence residual reaches tol, the true residual b - M x is
    recomputed; if it is still above tol (rounding drift at high viscosity
    contrast) CG restarts from x with it, within the same iteration budget.
    Returns (vx, vy, history): history[0] is the initial E_v and one entry
    follows per iteration (the last one the true E_v).  ``variants``: keyword
    arguments of ``vcycle_general`` (smoother variants) for the preconditioner."""
    L = levels[0]

    def vcycle(levels, l, vx, vy, bx, by, nu1, nu2, omega):
        if variants is None:
            return _vcycle_natural(levels, l, vx, vy, bx, by, nu1, nu2, omega)
        Lv = levels[l]
        x = SP.pack(Lv.nx, Lv.ny, vx, vy)
        c = -SP.pack(Lv.nx, Lv.ny, bx, by)
        return SP.unpack(Lv.nx, Lv.ny, vcycle_general(levels, l, x, c, nu1, nu2, omega, **variants))

    bx, by = S.rhs(L, fx, fy, p)
    dxg, dyg = S.diag(L)
    Nf = _masked_energy(fx, fy, dxg, dyg)
    if x0 is None:
        x = (np.zeros((L.ny, L.nx + 1)), np.zeros((L.ny + 1, L.nx)))
    else:
        x = (np.array(x0[0], float), np.array(x0[1], float))
    hist = []
    its = 0
    while True:
        mx, my = S.apply(L, *x)
        r = (bx - mx, by - my)                      # r = b - M x = -(residual of A x = -b)
        ev = np.sqrt(_masked_energy(r[0], r[1], dxg, dyg) / Nf)
        if hist:
            hist[-1] = ev
        else:
            hist.append(ev)
        if ev <= tol or its >= max_iters:
            return x[0], x[1], hist
        z = vcycle(levels, 0, np.zeros_like(bx), np.zeros_like(by), r[0], r[1], nu1, nu2, omega)  # ~ A^-1 (-r)
        pd = z
        gamma = -_dot(r, z)
        while its < max_iters:
            mp = S.apply(L, *pd)
            q = (-mp[0], -mp[1])                     # q = A p
            alpha = gamma / _dot(pd, q)
            x = (x[0] + alpha * pd[0], x[1] + alpha * pd[1])
            r_old = r
            r = (r[0] + alpha * q[0], r[1] + alpha * q[1])
            its += 1
            hist.append(np.sqrt(_masked_energy(r[0], r[1], dxg, dyg) / Nf))
            if hist[-1] <= tol:
                break
            z = vcycle(levels, 0, np.zeros_like(bx), np.zeros_like(by), r[0], r[1], nu1, nu2, omega)
            gamma_new = -_dot(r, z)
            beta = -_dot((r[0] - r_old[0], r[1] - r_old[1]), z) / gamma
            gamma = gamma_new
            pd = (z[0] + beta * pd[0], z[1] + beta * pd[1])
