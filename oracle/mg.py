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


def coarse_solve(L, bx, by):
    """Exact solution of M v = b on the coarsest level."""
    return SP.unpack(L.nx, L.ny, sla.cho_solve(L.chol, -SP.pack(L.nx, L.ny, bx, by)))


def _dot(a, b):
    return float(np.sum(a[0] * b[0]) + np.sum(a[1] * b[1]))


def _masked_energy(rx, ry, dxg, dyg):
    mx, my = dxg > 0, dyg > 0
    return float(np.sum(np.where(mx, rx * rx / np.where(mx, dxg, 1.0), 0.0)) +
                 np.sum(np.where(my, ry * ry / np.where(my, dyg, 1.0), 0.0)))


def pcg(levels, fx, fy, p=None, tol=1e-8, max_iters=500, nu1=2, nu2=2, omega=0.7, x0=None):
    """Flexible conjugate gradients on A x = -b (A = -M SPD, b = f - G p),
    preconditioned by one V-cycle per iteration, in FP64.  Stops when the
    velocity energy residual E_v = sqrt(N_v / N_f) of Sec. 6.4 is <= tol.
    When the recurrence residual reaches tol, the true residual b - M x is
    recomputed; if it is still above tol (rounding drift at high viscosity
    contrast) CG restarts from x with it, within the same iteration budget.
    Returns (vx, vy, history): history[0] is the initial E_v and one entry
    follows per iteration (the last one the true E_v)."""
    L = levels[0]
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
