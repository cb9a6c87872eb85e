"""FP64 geometric multigrid V-cycle and refinement loop (test infrastructure).

The paper solves the velocity block M v = f - G p with a matrix-free
geometric multigrid whose smoothing dominates the cost (Sec. 3.2, Sec. 5.2);
it does not print the transfer operators, the coarse viscosity rule or the
coarsest-grid solver.  This oracle takes the following reading:

  * coarsening by 2 in x and y down to ``coarsest`` cells (or an odd size);
  * coarse eta_c = mean of the 4 children, coarse eta_n = harmonic mean of the
    adjacent coarse cells; the coarse operator is rediscretised (p = 0);
  * bilinear prolongation P and restriction R = P^T/4 (``stokes_oracle.c``);
  * smoother S = damped Jacobi; RAS blocking with halo >= k-1 produces exactly
    Jacobi^k (Alg. 2 with enough overlap), so the oracle uses Jacobi^nu;
  * coarsest grid: exact FP64 solve (Cholesky of the assembled -M);
  * V(nu1, nu2): pre-smooth, residual, restrict, recurse from 0, prolong-add,
    post-smooth;
  * solve: V-cycle-preconditioned flexible conjugate gradients on the SPD
    system -M v = -b, stopping on the velocity energy residual
    E_v = sqrt(N_v/N_f) <= tol (Sec. 5.4).  A stand-alone V-cycle iteration
    with rediscretised coarse operators diverges once the viscosity contrast
    reaches ~1e3, so the correction solve is Krylov-accelerated (the paper's
    Anderson acceleration, Sec. 3.3 / Alg. 1, belongs to the same family).
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np
import scipy.linalg as sla

from . import stokes as S


def hierarchy(g, coarsest=16):
    levels = [SimpleNamespace(nx=g.nx, ny=g.ny, dx=g.dx, dy=g.dy, eta_c=np.asarray(g.eta_c, float),
                              eta_n=np.asarray(g.eta_n, float))]
    while True:
        L = levels[-1]
        if min(L.nx, L.ny) <= coarsest or L.nx % 2 or L.ny % 2:
            break
        ecc, enc = S.coarsen_eta(L)
        levels.append(SimpleNamespace(nx=L.nx // 2, ny=L.ny // 2, dx=2 * L.dx, dy=2 * L.dy, eta_c=ecc, eta_n=enc))
    _factor(levels[-1])
    return levels


def _unknown_index(L):
    mx = np.zeros((L.ny, L.nx + 1), dtype=bool)
    mx[:, 1:L.nx] = True
    my = np.zeros((L.ny + 1, L.nx), dtype=bool)
    my[1:L.ny, :] = True
    return mx, my


def _factor(L):
    """Assemble -M column by column (operator applied to unit vectors) and
    Cholesky-factor it."""
    mx, my = _unknown_index(L)
    ix, iy = np.flatnonzero(mx), np.flatnonzero(my)
    n = len(ix) + len(iy)
    A = np.zeros((n, n))
    for c in range(n):
        ex = np.zeros(mx.size)
        ey = np.zeros(my.size)
        if c < len(ix):
            ex[ix[c]] = 1.0
        else:
            ey[iy[c - len(ix)]] = 1.0
        ax, ay = S.apply(L, ex.reshape(mx.shape), ey.reshape(my.shape))
        A[:, c] = -np.concatenate([ax.ravel()[ix], ay.ravel()[iy]])
    L.A = A
    L.chol = sla.cho_factor(A)
    L.ix, L.iy = ix, iy


def coarse_solve(L, bx, by):
    """Exact solution of M v = b on the coarsest level (A v = -b)."""
    rhs = -np.concatenate([bx.ravel()[L.ix], by.ravel()[L.iy]])
    sol = sla.cho_solve(L.chol, rhs)
    vx = np.zeros((L.ny, L.nx + 1))
    vy = np.zeros((L.ny + 1, L.nx))
    vx.ravel()[L.ix] = sol[:len(L.ix)]
    vy.ravel()[L.iy] = sol[len(L.ix):]
    return vx, vy


def vcycle(levels, l, vx, vy, bx, by, nu1=2, nu2=2, omega=0.7):
    L = levels[l]
    if l == len(levels) - 1:
        return coarse_solve(L, bx, by)
    for _ in range(nu1):
        vx, vy = S.jacobi(L, bx, by, omega, vx, vy)
    mx, my = S.apply(L, vx, vy)
    rx, ry = bx - mx, by - my
    rx[:, 0] = rx[:, -1] = 0.0
    ry[0, :] = ry[-1, :] = 0.0
    cbx, cby = S.restrict(L.nx, L.ny, rx, ry)
    C = levels[l + 1]
    ex, ey = vcycle(levels, l + 1, np.zeros((C.ny, C.nx + 1)), np.zeros((C.ny + 1, C.nx)), cbx, cby,
                    nu1, nu2, omega)
    vx, vy = S.prolong_add(L.nx, L.ny, ex, ey, vx, vy)
    for _ in range(nu2):
        vx, vy = S.jacobi(L, bx, by, omega, vx, vy)
    return vx, vy


def _dot(a, b):
    return float(np.sum(a[0] * b[0]) + np.sum(a[1] * b[1]))


def _masked_energy(L, rx, ry, dxg, dyg):
    mx, my = dxg > 0, dyg > 0
    return float(np.sum(np.where(mx, rx * rx / np.where(mx, dxg, 1.0), 0.0)) +
                 np.sum(np.where(my, ry * ry / np.where(my, dyg, 1.0), 0.0)))


def pcg(levels, fx, fy, p=None, tol=1e-8, max_iters=500, nu1=2, nu2=2, omega=0.7, x0=None):
    """Flexible conjugate gradients on A x = -b (A = -M SPD, b = f - G p),
    preconditioned by one V-cycle per iteration, in FP64.  Stops when the
    velocity energy residual E_v = sqrt(N_v / N_f) of Sec. 5.4 is <= tol.
    Returns (vx, vy, history of E_v)."""
    L = levels[0]
    bx, by = S.rhs(L, fx, fy, p)
    dxg, dyg = S.diag(L)
    Nf = _masked_energy(L, fx, fy, dxg, dyg)
    if x0 is None:
        x = (np.zeros((L.ny, L.nx + 1)), np.zeros((L.ny + 1, L.nx)))
    else:
        x = (np.array(x0[0], float), np.array(x0[1], float))
    mx, my = S.apply(L, *x)
    r = (bx - mx, by - my)                      # r = b - M x = -(residual of A x = -b)
    hist = [np.sqrt(_masked_energy(L, r[0], r[1], dxg, dyg) / Nf)]
    if hist[-1] <= tol or max_iters == 0:
        return x[0], x[1], hist
    z = vcycle(levels, 0, np.zeros_like(bx), np.zeros_like(by), r[0], r[1], nu1, nu2, omega)  # ~ A^-1 (-r)
    pd = z
    gamma = -_dot(r, z)
    for it in range(max_iters):
        mp = S.apply(L, *pd)
        q = (-mp[0], -mp[1])                     # q = A p
        alpha = gamma / _dot(pd, q)
        x = (x[0] + alpha * pd[0], x[1] + alpha * pd[1])
        r_old = r
        r = (r[0] + alpha * q[0], r[1] + alpha * q[1])
        hist.append(np.sqrt(_masked_energy(L, r[0], r[1], dxg, dyg) / Nf))
        if hist[-1] <= tol or it == max_iters - 1:
            break
        z = vcycle(levels, 0, np.zeros_like(bx), np.zeros_like(by), r[0], r[1], nu1, nu2, omega)
        gamma_new = -_dot(r, z)
        beta = -_dot((r[0] - r_old[0], r[1] - r_old[1]), z) / gamma
        gamma = gamma_new
        pd = (z[0] + beta * pd[0], z[1] + beta * pd[1])
    return x[0], x[1], hist
