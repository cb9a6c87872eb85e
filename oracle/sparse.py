"""Sparse-matrix forms of the operator and the transfers (test infrastructure).

* ``operator_matrix(g)``: A = -M = B^T W B assembled as a scipy sparse matrix
  from the strain-rate form of the constitutive law (paper Sec. 2.1), the
  sparse twin of ``oracle.dense.assemble`` for grids of any size.
* ``prolongation_matrix(nx, ny)``: the bilinear prolongation P written from
  its weights (normal axis: 1 on coinciding faces, 1/2 between faces;
  tangential axis: 3/4 on the own coarse row, 1/4 on the neighbour row,
  mirrored at the free-slip walls).

Unknowns are numbered as in ``oracle.dense.Dofs``: vx(i,j) (1<=i<=nx-1,
0<=j<ny) row-major, then vy(i,j) (0<=i<nx, 1<=j<=ny-1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def numbering(nx, ny):
    """(index arrays) nvx, vx_id[j, i] (-1 on walls), vy_id[j, i]."""
    vx_id = -np.ones((ny, nx + 1), dtype=np.int64)
    vx_id[:, 1:nx] = np.arange(ny * (nx - 1)).reshape(ny, nx - 1)
    nvx = ny * (nx - 1)
    vy_id = -np.ones((ny + 1, nx), dtype=np.int64)
    vy_id[1:ny, :] = nvx + np.arange((ny - 1) * nx).reshape(ny - 1, nx)
    return nvx, vx_id, vy_id


def n_unknowns(nx, ny):
    return ny * (nx - 1) + (ny - 1) * nx


def pack(nx, ny, vx, vy):
    return np.concatenate([np.asarray(vx)[:, 1:nx].ravel(), np.asarray(vy)[1:ny, :].ravel()])


def unpack(nx, ny, v):
    vx = np.zeros((ny, nx + 1))
    vy = np.zeros((ny + 1, nx))
    nvx = ny * (nx - 1)
    vx[:, 1:nx] = v[:nvx].reshape(ny, nx - 1)
    vy[1:ny, :] = v[nvx:].reshape(ny - 1, nx)
    return vx, vy


def strain_matrix(nx, ny, dx, dy):
    """B: rows exx per cell, eyy per cell, gxy per interior node."""
    _, vx_id, vy_id = numbering(nx, ny)
    rows, cols, vals = [], [], []

    def add(r, ids, v):
        m = ids >= 0
        rows.append(r[m])
        cols.append(ids[m])
        vals.append(np.broadcast_to(v, ids.shape)[m])

    nc = nx * ny
    r_exx = np.arange(nc).reshape(ny, nx)
    add(r_exx, vx_id[:, 1:], 1.0 / dx)
    add(r_exx, vx_id[:, :-1], -1.0 / dx)
    r_eyy = nc + np.arange(nc).reshape(ny, nx)
    add(r_eyy, vy_id[1:, :], 1.0 / dy)
    add(r_eyy, vy_id[:-1, :], -1.0 / dy)
    r_g = 2 * nc + np.arange((nx - 1) * (ny - 1)).reshape(ny - 1, nx - 1)  # node (i,j), 1<=i,j
    add(r_g, vx_id[1:ny, 1:nx], 1.0 / dy)       # vx(i, j)
    add(r_g, vx_id[0:ny - 1, 1:nx], -1.0 / dy)  # vx(i, j-1)
    add(r_g, vy_id[1:ny, 1:nx], 1.0 / dx)       # vy(i, j)
    add(r_g, vy_id[1:ny, 0:nx - 1], -1.0 / dx)  # vy(i-1, j)
    nrow = 2 * nc + (nx - 1) * (ny - 1)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nrow, n_unknowns(nx, ny)))


def operator_matrix(g):
    """A = -M = B^T W B, W = diag(2 eta_c, 2 eta_c, eta_n at interior nodes)."""
    B = strain_matrix(g.nx, g.ny, g.dx, g.dy)
    ec = np.asarray(g.eta_c, float).ravel()
    en = np.asarray(g.eta_n, float)[1:g.ny, 1:g.nx].ravel()
    w = np.concatenate([2 * ec, 2 * ec, en])
    return (B.T @ sp.diags(w) @ B).tocsr()


def _axis(nf, nc, normal):
    """1-D weight matrix (nf x nc positions) of one axis."""
    rows, cols, vals = [], [], []
    for f in range(nf):
        if normal:
            if f % 2 == 0:
                rows.append(f); cols.append(f // 2); vals.append(1.0)
            else:
                rows += [f, f]; cols += [(f - 1) // 2, (f + 1) // 2]; vals += [0.5, 0.5]
        else:
            J = f // 2
            nb = J + 1 if f % 2 else J - 1
            if nb < 0 or nb >= nc:
                rows.append(f); cols.append(J); vals.append(1.0)
            else:
                rows += [f, f]; cols += [J, nb]; vals += [0.75, 0.25]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def prolongation_matrix(nx, ny):
    """P (fine unknowns x coarse unknowns) for a fine grid nx x ny (even)."""
    NX, NY = nx // 2, ny // 2
    # vx: x axis normal (faces 0..nx / 0..NX), y axis tangential (rows)
    Px = sp.kron(_axis(ny, NY, False), _axis(nx + 1, NX + 1, True)).tocsr()
    Py = sp.kron(_axis(ny + 1, NY + 1, True), _axis(nx, NX, False)).tocsr()
    # restrict to unknowns (walls are not unknowns; coarse walls carry 0)
    fx = np.zeros((ny, nx + 1), bool); fx[:, 1:nx] = True
    cx = np.zeros((NY, NX + 1), bool); cx[:, 1:NX] = True
    fy = np.zeros((ny + 1, nx), bool); fy[1:ny, :] = True
    cy = np.zeros((NY + 1, NX), bool); cy[1:NY, :] = True
    Px = Px[np.flatnonzero(fx.ravel())][:, np.flatnonzero(cx.ravel())]
    Py = Py[np.flatnonzero(fy.ravel())][:, np.flatnonzero(cy.ravel())]
    return sp.block_diag([Px, Py]).tocsr()
