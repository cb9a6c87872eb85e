"""Pins of the CPU oracle's discrete operator (no GPU).

The paper prints no worked numbers, so the oracle is pinned by what the
mathematics fixes: a manufactured solution (continuum operator from sympy,
second-order consistency), a closed-form discrete eigenmode, an independent
assembly A = B^T W B from the energy form, symmetry/definiteness (Sec. 6.4:
M symmetric negative definite), G = D^T, and hydrostatic balance.
"""
from types import SimpleNamespace

import numpy as np
import pytest
import sympy as sp

from oracle import dense as Dn
from oracle import stokes as S


def grid(nx, ny, eta_c, eta_n, dx=None, dy=None):
    return SimpleNamespace(nx=nx, ny=ny, dx=dx or 1.0 / nx, dy=dy or 1.0 / ny, eta_c=eta_c, eta_n=eta_n)


def rand_grid(nx, ny, seed, lo=-1.0, hi=2.0, dx=None, dy=None):
    rng = np.random.default_rng(seed)
    return grid(nx, ny, 10 ** rng.uniform(lo, hi, (ny, nx)), 10 ** rng.uniform(lo, hi, (ny + 1, nx + 1)), dx, dy)


def rand_v(nx, ny, seed):
    rng = np.random.default_rng(seed)
    vx, vy = rng.standard_normal((ny, nx + 1)), rng.standard_normal((ny + 1, nx))
    vx[:, [0, -1]] = 0.0
    vy[[0, -1], :] = 0.0
    return vx, vy


# ------------------------------------------------------------------ sympy --
_x, _y = sp.symbols("x y")
_eta = sp.exp(sp.sin(2 * sp.pi * _x) * sp.cos(sp.pi * _y))
# vx = 0 on x = 0, 1; vy = 0 on y = 0, 1; shear vanishes on every wall
_vx = sp.sin(sp.pi * _x) * sp.cos(sp.pi * _y) + sp.Rational(3, 10) * sp.sin(2 * sp.pi * _x) * sp.cos(3 * sp.pi * _y)
_vy = sp.Rational(1, 2) * sp.cos(sp.pi * _x) * sp.sin(sp.pi * _y) + sp.Rational(1, 5) * sp.cos(3 * sp.pi * _x) * sp.sin(2 * sp.pi * _y)
_p = sp.cos(sp.pi * _x) * sp.sin(2 * sp.pi * _y)
_txy = _eta * (sp.diff(_vx, _y) + sp.diff(_vy, _x))
# Cauchy form, Sec. 2.1: d(sigma'_xx)/dx + d(sigma'_xy)/dy and its y twin
_Mx = sp.diff(2 * _eta * sp.diff(_vx, _x), _x) + sp.diff(_txy, _y)
_My = sp.diff(_txy, _x) + sp.diff(2 * _eta * sp.diff(_vy, _y), _y)
_div = sp.diff(_vx, _x) + sp.diff(_vy, _y)
F = {k: sp.lambdify((_x, _y), e, "numpy") for k, e in
     dict(eta=_eta, vx=_vx, vy=_vy, Mx=_Mx, My=_My, div=_div, p=_p, px=sp.diff(_p, _x), py=sp.diff(_p, _y)).items()}


def manufactured(nx, ny):
    dx, dy = 1.0 / nx, 1.0 / ny
    xc, yc = (np.arange(nx) + 0.5) * dx, (np.arange(ny) + 0.5) * dy
    xn, yn = np.arange(nx + 1) * dx, np.arange(ny + 1) * dy
    g = grid(nx, ny, F["eta"](*np.meshgrid(xc, yc)), F["eta"](*np.meshgrid(xn, yn)))
    VX = np.meshgrid(xn, yc)  # vx points
    VY = np.meshgrid(xc, yn)  # vy points
    vx, vy = F["vx"](*VX), F["vy"](*VY)
    vx[:, [0, -1]] = 0.0
    vy[[0, -1], :] = 0.0
    return g, VX, VY, vx, vy, np.meshgrid(xc, yc)


@pytest.mark.parametrize("aspect", [1, 2])
def test_operator_second_order_consistent_with_continuum(aspect):
    """Stencil applied to a sampled smooth field vs the continuum operator with
    variable viscosity: error O(h^2) (wrong sign, index or eta placement would
    give O(1) or O(h))."""
    errs = []
    for n in (16, 32, 64):
        g, VX, VY, vx, vy, _ = manufactured(aspect * n, n)
        mx, my = S.apply(g, vx, vy)
        ex = np.abs(mx[:, 1:-1] - F["Mx"](*VX)[:, 1:-1]).max()
        ey = np.abs(my[1:-1, :] - F["My"](*VY)[1:-1, :]).max()
        errs.append(max(ex, ey))
    scale = np.abs(F["Mx"](*manufactured(64, 64)[1])).max()
    assert errs[-1] < 2e-2 * scale
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_divergence_and_pressure_gradient_second_order():
    e_div, e_gp = [], []
    for n in (16, 32, 64):
        g, VX, VY, vx, vy, C = manufactured(n, n)
        e_div.append(np.abs(S.divergence(g, vx, vy) - F["div"](*C)).max())
        p = F["p"](*C)
        # b - f = -G p approximates grad p at the velocity points
        bx, by = S.rhs(g, np.zeros_like(vx), np.zeros_like(vy), p)
        e_gp.append(max(np.abs(bx[:, 1:-1] - F["px"](*VX)[:, 1:-1]).max(),
                        np.abs(by[1:-1] - F["py"](*VY)[1:-1]).max()))
    for e in (e_div, e_gp):
        assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, e


@pytest.mark.parametrize("n,dx,dy", [(32, None, None), (48, None, None), (24, 1 / 24, 1 / 40)])
def test_constant_viscosity_closed_form(n, dx, dy):
    """Constant eta: vx = sin(pi x)cos(pi y), vy = c cos(pi x) sin(pi y) with c
    chosen so the discrete shear vanishes; then (-M v)_x = 8 eta sin^2(pi dx/2)/dx^2 vx
    and (-M v)_y = 8 eta sin^2(pi dy/2)/dy^2 vy exactly (dx = dy: an eigenmode)."""
    eta = 3.0
    dx = dx or 1.0 / n
    dy = dy or 1.0 / n
    ny = int(round(1 / dy))
    g = grid(n, ny, np.full((ny, n), eta), np.full((ny + 1, n + 1), eta), dx, dy)
    xn, yc = np.arange(n + 1) * dx, (np.arange(ny) + 0.5) * dy
    xc, yn = (np.arange(n) + 0.5) * dx, np.arange(ny + 1) * dy
    c = -(np.sin(np.pi * dy / 2) / dy) / (np.sin(np.pi * dx / 2) / dx)
    vx = np.sin(np.pi * xn)[None, :] * np.cos(np.pi * yc)[:, None]
    vy = c * np.cos(np.pi * xc)[None, :] * np.sin(np.pi * yn)[:, None]
    vx[:, [0, -1]] = 0.0
    vy[[0, -1], :] = 0.0
    mx, my = S.apply(g, vx, vy)
    lx = 8 * eta * np.sin(np.pi * dx / 2) ** 2 / dx ** 2
    ly = 8 * eta * np.sin(np.pi * dy / 2) ** 2 / dy ** 2
    assert np.abs(-mx - lx * vx).max() <= 1e-12 * lx
    assert np.abs(-my - ly * vy).max() <= 1e-12 * ly
    # discrete divergence of the dx = dy mode is zero
    if dx == dy:
        assert np.abs(S.divergence(g, vx, vy)).max() <= 1e-12 / dx


@pytest.mark.parametrize("nx,ny,dx,dy,seed", [(4, 3, None, None, 0), (7, 5, None, None, 1), (8, 8, 0.3, 0.7, 2),
                                              (2, 6, None, None, 3), (6, 2, 0.11, 0.05, 4)])
def test_stencil_equals_assembled_BtWB(nx, ny, dx, dy, seed):
    g = rand_grid(nx, ny, seed, dx=dx, dy=dy)
    A, d = Dn.assemble(g)
    vx, vy = rand_v(nx, ny, seed + 10)
    mx, my = S.apply(g, vx, vy)
    Av = A @ d.pack(vx, vy)
    assert np.abs(d.pack(-mx, -my) - Av).max() <= 1e-13 * np.abs(Av).max()
    dxg, dyg = S.diag(g)
    assert np.abs(d.pack(dxg, dyg) - np.diag(A)).max() <= 1e-13 * np.abs(np.diag(A)).max()
    # the walls are not part of the state: garbage there changes nothing
    vx2, vy2 = vx.copy(), vy.copy()
    vx2[:, [0, -1]] = 123.0
    vy2[[0, -1], :] = -7.0
    mx2, my2 = S.apply(g, vx2, vy2)
    assert np.array_equal(mx, mx2) and np.array_equal(my, my2)


def test_symmetric_negative_definite():
    """Sec. 6.4: M is symmetric negative definite under these BCs."""
    g = rand_grid(37, 29, 5, lo=-2, hi=4)
    u = rand_v(37, 29, 6)
    v = rand_v(37, 29, 7)
    Mu, Mv = S.apply(g, *u), S.apply(g, *v)
    a = np.sum(Mu[0] * v[0]) + np.sum(Mu[1] * v[1])
    b = np.sum(u[0] * Mv[0]) + np.sum(u[1] * Mv[1])
    scale = np.sqrt((np.sum(Mu[0] ** 2) + np.sum(Mu[1] ** 2)) * (np.sum(v[0] ** 2) + np.sum(v[1] ** 2)))
    assert abs(a - b) <= 1e-13 * scale
    assert -(np.sum(Mu[0] * u[0]) + np.sum(Mu[1] * u[1])) > 0
    A, _ = Dn.assemble(rand_grid(6, 5, 8, lo=-3, hi=3))
    assert np.linalg.eigvalsh(A).min() > 0


def test_gradient_is_divergence_transpose():
    """<G p, v> = <p, D v> with G p = -(b - f) from the RHS fold."""
    g = rand_grid(13, 11, 9)
    rng = np.random.default_rng(10)
    p = rng.standard_normal((11, 13))
    vx, vy = rand_v(13, 11, 11)
    bx, by = S.rhs(g, np.zeros((11, 14)), np.zeros((12, 13)), p)
    lhs = -(np.sum(bx * vx) + np.sum(by * vy))
    rhs = np.sum(p * S.divergence(g, vx, vy))
    assert abs(lhs - rhs) <= 1e-12 * np.abs(p).sum() * 13
    # and the assembled D agrees with the stencil divergence
    A, d = Dn.assemble(g)
    Dm = Dn.divergence_matrix(g, d)
    assert np.allclose(Dm @ d.pack(vx, vy), S.divergence(g, vx, vy).ravel(), rtol=0, atol=1e-10)


def test_hydrostatic_pressure_balances_gravity():
    """Constant density rho, gravity -y, fy = rho |g|: the lithostatic
    pressure p = -rho y (Sec. 6.2, integral of rho g) gives b = f - G p = 0."""
    nx, ny, rho = 10, 12, 1.3
    g = rand_grid(nx, ny, 12)
    yc = (np.arange(ny) + 0.5) / ny
    p = np.repeat((-rho * yc)[:, None], nx, axis=1)
    bx, by = S.rhs(g, np.zeros((ny, nx + 1)), np.full((ny + 1, nx), rho), p)
    assert np.abs(bx).max() <= 1e-13 and np.abs(by).max() <= 1e-12
