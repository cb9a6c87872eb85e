"""Device layout helpers: natural numpy fields <-> padded device tensors.

The library's layout is row-major with one common row stride ``ld`` for all
fields (include/stk.h).  Here every field is held in a (ny+1) x ld tensor,
``ld`` = nx+1 rounded up to a multiple of 64 elements so rows start on
256/512-byte boundaries.  Pure data movement, no arithmetic of the method.
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import Grid, Grid3


def pad_ld(nx: int, align: int = 64) -> int:
    return ((nx + 1 + align - 1) // align) * align


def upload(a: np.ndarray, rows: int, ld: int, dtype, device="cuda") -> torch.Tensor:
    t = torch.zeros((rows, ld), dtype=dtype)
    t[: a.shape[0], : a.shape[1]] = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dtype)
    return t.to(device)


def download(t: torch.Tensor, shape) -> np.ndarray:
    return t[: shape[0], : shape[1]].to(torch.float64).cpu().numpy()


class DeviceProblem:
    """A problem's eta_c, eta_n, fx, fy on the device in the stk layout."""

    def __init__(self, prob, dtype=torch.float64, device="cuda", align: int = 64):
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        self.ld = pad_ld(prob.nx, align)
        self.dtype = dtype
        self.device = device
        self.grid = Grid(prob.nx, prob.ny, self.ld, float(prob.dx), float(prob.dy))
        R = prob.ny + 1
        self.eta_c = upload(prob.eta_c, R, self.ld, dtype, device)
        self.eta_n = upload(prob.eta_n, R, self.ld, dtype, device)
        self.fx = upload(prob.fx, R, self.ld, dtype, device)
        self.fy = upload(prob.fy, R, self.ld, dtype, device)

    @property
    def shape_vx(self):
        return (self.ny, self.nx + 1)

    @property
    def shape_vy(self):
        return (self.ny + 1, self.nx)

    def field(self, a=None):
        """A zero (ny+1) x ld tensor, optionally filled with natural array ``a``."""
        if a is None:
            return torch.zeros((self.ny + 1, self.ld), dtype=self.dtype, device=self.device)
        return upload(a, self.ny + 1, self.ld, self.dtype, self.device)

    def velocity(self, vx=None, vy=None):
        return self.field(vx), self.field(vy)

    def get_vx(self, t):
        return download(t, self.shape_vx)

    def get_vy(self, t):
        return download(t, self.shape_vy)

    def get_cell(self, t):
        return download(t, (self.ny, self.nx))


class DeviceProblem3:
    """A 3D problem's viscosities and right-hand side on the device: every field
    (nz+1) x (ny+1) x ld, plane stride lp = (ny+1) ld."""

    def __init__(self, prob, dtype=torch.float64, device="cuda", align: int = 64):
        self.prob = prob
        self.nx, self.ny, self.nz = prob.nx, prob.ny, prob.nz
        self.ld = pad_ld(prob.nx, align)
        self.lp = (prob.ny + 1) * self.ld
        self.dtype, self.device = dtype, device
        self.grid = Grid3(prob.nx, prob.ny, prob.nz, self.ld, self.lp, float(prob.dx), float(prob.dy),
                          float(prob.dz))
        self.eta = tuple(self.field(a) for a in (prob.eta_c, prob.eta_xy, prob.eta_xz, prob.eta_yz))
        self.f = tuple(self.field(a) for a in (prob.fx, prob.fy, prob.fz))

    def field(self, a=None):
        t = torch.zeros((self.nz + 1, self.ny + 1, self.ld), dtype=self.dtype)
        if a is not None:
            t[: a.shape[0], : a.shape[1], : a.shape[2]] = torch.from_numpy(
                np.ascontiguousarray(a, dtype=np.float64)).to(self.dtype)
        return t.to(self.device)

    def velocity(self, v=None):
        return tuple(self.field(None if v is None else a) for a in (v if v is not None else (None, None, None)))

    def get(self, t, shape):
        return t[: shape[0], : shape[1], : shape[2]].to(torch.float64).cpu().numpy()

    def get_v(self, v):
        nx, ny, nz = self.nx, self.ny, self.nz
        return (self.get(v[0], (nz, ny, nx + 1)), self.get(v[1], (nz, ny + 1, nx)), self.get(v[2], (nz + 1, ny, nx)))

