"""Assembled-matrix oracle for tiny grids (test infrastructure only).

An independent route to the discrete velocity operator: the energy form of
the constitutive law (paper Sec. 2.1, sigma' = 2 eta strain-rate) gives
A = -M = B^T W B, where B maps velocities to the strain-rate rows

    exx(i,j) = (vx(i+1,j)-vx(i,j))/dx          one row per cell
    eyy(i,j) = (vy(i,j+1)-vy(i,j))/dy          one row per cell
    gxy(i,j) = (vx(i,j)-vx(i,j-1))/dy + (vy(i,j)-vy(i-1,j))/dx
                                               one row per interior node

and W = diag(2 eta_c, 2 eta_c, eta_n).  Wall velocities are not unknowns
(Dirichlet 0); boundary nodes carry no shear row (free slip).  Nothing here
calls the stencil code in ``stokes_oracle.c``.
"""
from __future__ import annotations

import numpy as np


class Dofs:
    """Numbering of the unknowns: vx(i,j), 1<=i<=nx-1, 0<=j<ny, then
    vy(i,j), 0<=i<nx, 1<=j<=ny-1 (row-major in j, then i)."""

    def __init__(self, nx, ny):
        self.nx, self.ny = nx, ny
        self.vx = {}
        self.vy = {}
        k = 0
        for j in range(ny):
            for i in range(1, nx):
                self.vx[(i, j)] = k
                k += 1
        for j in range(1, ny):
            for i in range(nx):
                self.vy[(i, j)] = k
                k += 1
        self.n = k

    def pack(self, vx, vy):
        v = np.zeros(self.n)
        for (i, j), k in self.vx.items():
            v[k] = vx[j, i]
        for (i, j), k in self.vy.items():
            v[k] = vy[j, i]
        return v

    def unpack(self, v):
        vx = np.zeros((self.ny, self.nx + 1))
        vy = np.zeros((self.ny + 1, self.nx))
        for (i, j), k in self.vx.items():
            vx[j, i] = v[k]
        for (i, j), k in self.vy.items():
            vy[j, i] = v[k]
        return vx, vy

    def cell_of(self):
        """Cell (i,j) that each unknown belongs to (its left vx / bottom vy)."""
        c = [None] * self.n
        for (i, j), k in self.vx.items():
            c[k] = (i, j)
        for (i, j), k in self.vy.items():
            c[k] = (i, j)
        return c

    def colour(self):
        """Red-black colour (i+j) mod 2 and component (0 = vx, 1 = vy)."""
        col = np.zeros(self.n, dtype=int)
        comp = np.zeros(self.n, dtype=int)
        for (i, j), k in self.vx.items():
            col[k] = (i + j) % 2
        for (i, j), k in self.vy.items():
            col[k] = (i + j) % 2
            comp[k] = 1
        return col, comp


def strain_matrix(nx, ny, dx, dy, dofs=None):
    """B and the row weights' sources: returns (B, kinds, where)."""
    d = dofs or Dofs(nx, ny)
    rows = []
    kinds = []
    where = []

    def vx_col(i, j):
        return d.vx.get((i, j))

    def vy_col(i, j):
        return d.vy.get((i, j))

    for j in range(ny):
        for i in range(nx):
            r = np.zeros(d.n)
            for (ii, s) in ((i + 1, 1.0), (i, -1.0)):
                c = vx_col(ii, j)
                if c is not None:
                    r[c] += s / dx
            rows.append(r); kinds.append("c"); where.append((i, j))
            r = np.zeros(d.n)
            for (jj, s) in ((j + 1, 1.0), (j, -1.0)):
                c = vy_col(i, jj)
                if c is not None:
                    r[c] += s / dy
            rows.append(r); kinds.append("c"); where.append((i, j))
    for j in range(1, ny):
        for i in range(1, nx):
            r = np.zeros(d.n)
            for (jj, s) in ((j, 1.0), (j - 1, -1.0)):
                c = vx_col(i, jj)
                if c is not None:
                    r[c] += s / dy
            for (ii, s) in ((i, 1.0), (i - 1, -1.0)):
                c = vy_col(ii, j)
                if c is not None:
                    r[c] += s / dx
            rows.append(r); kinds.append("n"); where.append((i, j))
    return np.array(rows), kinds, where


def assemble(g):
    """A = -M = B^T W B as a dense (n x n) matrix, plus the numbering."""
    d = Dofs(g.nx, g.ny)
    B, kinds, where = strain_matrix(g.nx, g.ny, g.dx, g.dy, d)
    w = np.array([2.0 * g.eta_c[j, i] if k == "c" else g.eta_n[j, i] for k, (i, j) in zip(kinds, where)])
    return B.T @ (w[:, None] * B), d


def divergence_matrix(g, dofs=None):
    """D (cells x unknowns): (Dv)(i,j) = (vx(i+1,j)-vx(i,j))/dx + (vy(i,j+1)-vy(i,j))/dy."""
    d = dofs or Dofs(g.nx, g.ny)
    Dm = np.zeros((g.nx * g.ny, d.n))
    for j in range(g.ny):
        for i in range(g.nx):
            row = j * g.nx + i
            for (ii, s) in ((i + 1, 1.0), (i, -1.0)):
                c = d.vx.get((ii, j))
                if c is not None:
                    Dm[row, c] += s / g.dx
            for (jj, s) in ((j + 1, 1.0), (j, -1.0)):
                c = d.vy.get((i, jj))
                if c is not None:
                    Dm[row, c] += s / g.dy
    return Dm


# ---------------------------------------------------------------- smoothers --
# All in terms of A = -M: M v = b  <=>  A v = -b, residual b - M v = b + A v.

def jacobi(A, b, v, omega):
    return v - omega * (b + A @ v) / np.diag(A)


def rbgs(A, b, v, omega, dofs):
    """Set-ordered Gauss-Seidel: vx-red, vx-black, vy-red, vy-black."""
    col, comp = dofs.colour()
    v = v.copy()
    dA = np.diag(A)
    for c in (0, 1):
        for k in (0, 1):
            S = (comp == c) & (col == k)
            r = b + A @ v
            v[S] = v[S] - omega * r[S] / dA[S]
    return v


def _cuts(n, T, s):
    s %= T
    out = []
    t = 0
    while True:
        a, b = max(0, s + (t - 1) * T), min(n, s + t * T)
        if a >= n:
            break
        if a < b:
            out.append((a, b))
        t += 1
    return out


def ras_outer(A, b, u, omega, dofs, Tx, Ty, h, kt, sx, sy):
    """RAS outer iteration as a per-tile subdomain problem: on the extended
    unknown set E (cells within h of the tile, clipped), run kt Jacobi steps
    for A_EE w = -b_E - A_{E,rest} u_rest (Dirichlet data u outside E), then
    keep the owned unknowns."""
    nx, ny = dofs.nx, dofs.ny
    cells = dofs.cell_of()
    out = u.copy()
    for (x0, x1) in _cuts(nx, Tx, sx):
        for (y0, y1) in _cuts(ny, Ty, sy):
            X0, X1, Y0, Y1 = max(0, x0 - h), min(nx, x1 + h), max(0, y0 - h), min(ny, y1 + h)
            E = np.array([X0 <= ci <= X1 - 1 and Y0 <= cj <= Y1 - 1 for (ci, cj) in cells])
            own = np.array([x0 <= ci <= x1 - 1 and y0 <= cj <= y1 - 1 for (ci, cj) in cells])
            R = ~E
            AEE = A[np.ix_(E, E)]
            rhs = -b[E] - A[np.ix_(E, R)] @ u[R]
            w = u[E].copy()
            dE = np.diag(AEE)
            for _ in range(kt):
                w = w - omega * (AEE @ w - rhs) / dE
            full = u.copy()
            full[E] = w
            out[own] = full[own]
    return out
