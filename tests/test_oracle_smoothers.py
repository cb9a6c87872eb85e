"""Pins of the oracle's smoothers, RAS blocking and energy norm (no GPU).

Jacobi and red-black Gauss-Seidel are checked against textbook dense-matrix
iterations on the independently assembled A = B^T W B; RAS-type temporal
blocking (Alg. 2, snapshot semantics) against Jacobi^k where the overlap makes
them identical and against a dense per-tile subdomain formulation where it
does not; the energy norm (Sec. 6.4) against its exact special cases.
"""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import dense as Dn
from oracle import mg
from oracle import stokes as S
from paper_2509_19061_amd import inputs as I


def rand_problem(nx, ny, seed, lo=-1.0, hi=3.0):
    rng = np.random.default_rng(seed)
    g = SimpleNamespace(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / ny, eta_c=10 ** rng.uniform(lo, hi, (ny, nx)))
    g.eta_n = I.nodal_harmonic(g.eta_c)
    bx, by = rng.standard_normal((ny, nx + 1)), rng.standard_normal((ny + 1, nx))
    bx[:, [0, -1]] = 0.0
    by[[0, -1], :] = 0.0
    vx, vy = I.random_velocity(g, seed + 1)
    return g, bx, by, vx, vy


@pytest.mark.parametrize("nx,ny,omega", [(5, 4, 0.7), (8, 8, 0.6), (3, 7, 1.0)])
def test_jacobi_and_rbgs_equal_dense_iterations(nx, ny, omega):
    g, bx, by, vx, vy = rand_problem(nx, ny, nx * 10 + ny)
    A, d = Dn.assemble(g)
    b, v = d.pack(bx, by), d.pack(vx, vy)
    jx, jy = S.jacobi(g, bx, by, omega, vx, vy)
    ref = Dn.jacobi(A, b, v, omega)
    assert np.abs(d.pack(jx, jy) - ref).max() <= 1e-12 * np.abs(ref).max()
    rx, ry = S.rbgs(g, bx, by, omega, vx, vy)
    ref = Dn.rbgs(A, b, v, omega, d)
    assert np.abs(d.pack(rx, ry) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_rbgs_sets_do_not_couple():
    """Within one colour set of one component the unknowns do not couple, so
    a set-ordered sweep is well defined (red-black premise, Sec. 4 (i))."""
    g, *_ = rand_problem(7, 6, 3)
    A, d = Dn.assemble(g)
    col, comp = d.colour()
    for c in (0, 1):
        for k in (0, 1):
            Sset = (comp == c) & (col == k)
            blk = A[np.ix_(Sset, Sset)]
            assert np.abs(blk - np.diag(np.diag(blk))).max() == 0.0


def test_ras_single_tile_is_jacobi():
    """One tile covering the domain: RAS = Jacobi^k, bit for bit."""
    g, bx, by, vx, vy = rand_problem(20, 17, 4)
    ox, oy = S.ras_outer(g, bx, by, 0.7, 64, 64, 0, 3, 0, 0, vx, vy)
    jx, jy = vx, vy
    for _ in range(3):
        jx, jy = S.jacobi(g, bx, by, 0.7, jx, jy)
    assert np.array_equal(ox, jx) and np.array_equal(oy, jy)


@pytest.mark.parametrize("T,k,h,sx,sy", [(8, 4, 3, 0, 0), (8, 4, 4, 5, 2), (5, 3, 2, 4, 1), (6, 1, 0, 3, 5),
                                         (7, 2, 1, 6, 6), (4, 5, 4, 1, 3)])
def test_ras_with_overlap_at_least_k_minus_1_is_jacobi(T, k, h, sx, sy):
    """Frozen values outside the extended tile reach at most k-1 cells inward
    after k sweeps, so halo >= k-1 reproduces Jacobi^k exactly for any tile
    size and shift; k = 1, h = 0 is the blocked fused Jacobi."""
    g, bx, by, vx, vy = rand_problem(23, 19, 5)
    ox, oy = S.ras_outer(g, bx, by, 0.7, T, T, h, k, sx, sy, vx, vy)
    jx, jy = vx, vy
    for _ in range(k):
        jx, jy = S.jacobi(g, bx, by, 0.7, jx, jy)
    assert np.array_equal(ox, jx) and np.array_equal(oy, jy)


def test_ras_with_thin_overlap_differs_from_jacobi():
    g, bx, by, vx, vy = rand_problem(23, 19, 6)
    ox, oy = S.ras_outer(g, bx, by, 0.7, 6, 6, 1, 4, 2, 3, vx, vy)
    jx, jy = vx, vy
    for _ in range(4):
        jx, jy = S.jacobi(g, bx, by, 0.7, jx, jy)
    assert np.abs(ox - jx).max() > 1e-6


@pytest.mark.parametrize("nx,ny,T,h,k,sx,sy", [(9, 8, 4, 0, 3, 1, 2), (10, 7, 3, 1, 4, 2, 0), (8, 8, 5, 0, 2, 0, 4),
                                               (11, 9, 4, 2, 5, 3, 3)])
def test_ras_equals_dense_subdomain_solves(nx, ny, T, h, k, sx, sy):
    """Alg. 2 read as restricted additive Schwarz: each tile solves its
    extended subdomain with Dirichlet data from the snapshot outside it, by k
    Jacobi steps, and keeps its owned unknowns (dense formulation)."""
    g, bx, by, vx, vy = rand_problem(nx, ny, nx + ny + T)
    A, d = Dn.assemble(g)
    ref = Dn.ras_outer(A, d.pack(bx, by), d.pack(vx, vy), 0.7, d, T, T, h, k, sx, sy)
    ox, oy = S.ras_outer(g, bx, by, 0.7, T, T, h, k, sx, sy, vx, vy)
    assert np.abs(d.pack(ox, oy) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_ras_rectangular_tiles_and_partial_last_outer():
    g, bx, by, vx, vy = rand_problem(17, 13, 7)
    A, d = Dn.assemble(g)
    shifts = [(3, 1), (0, 4), (5, 2)]
    ks = S.n_outer(10, 4)
    assert ks == [4, 4, 2]
    assert S.n_outer(10, 4, last_partial=False) == [4, 4, 4]
    ref = d.pack(vx, vy)
    b = d.pack(bx, by)
    for (sx, sy), kt in zip(shifts, ks):
        ref = Dn.ras_outer(A, b, ref, 0.7, d, 6, 4, 1, kt, sx, sy)
    ox, oy = vx, vy
    for (sx, sy), kt in zip(shifts, ks):
        ox, oy = S.ras_outer(g, bx, by, 0.7, 6, 4, 1, kt, sx, sy, ox, oy)
    assert np.abs(d.pack(ox, oy) - ref).max() <= 1e-12 * np.abs(ref).max()


# ----------------------------------------------------------- energy norm --

def test_energy_norm_of_zero_state_is_one():
    """v = 0, p = 0: r_v = f, r_p = 0, so E = E_v = 1 exactly (Sec. 6.4)."""
    p = I.random_sinkers(48, 3, 1, eta_in=1e4)
    out = S.energy(p, *p.zeros_v(), p.fx, p.fy)
    assert out[1] == 0.0 and out[0] == out[2] and out[3] == 1.0 and out[4] == 1.0


def test_energy_norm_pieces_against_dense():
    g, bx, by, vx, vy = rand_problem(7, 6, 8)
    rng = np.random.default_rng(9)
    fx, fy = bx, by
    p = rng.standard_normal((6, 7))
    A, d = Dn.assemble(g)
    Dm = Dn.divergence_matrix(g, d)
    v = d.pack(vx, vy)
    # b = f - G p with G = D^T (dense), r_v = b - M v = b + A v
    b = d.pack(fx, fy) - Dm.T @ p.ravel()
    rv = b + A @ v
    rp = -(Dm @ v)
    dA = np.diag(A)
    Nv = np.sum(rv ** 2 / dA)
    Np = np.sum(rp ** 2 * g.eta_c.ravel() / (2 / g.dx ** 2 + 2 / g.dy ** 2))
    Nf = np.sum(d.pack(fx, fy) ** 2 / dA)
    out = S.energy(g, vx, vy, fx, fy, p)
    np.testing.assert_allclose(out[:3], [Nv, Np, Nf], rtol=1e-12)
    np.testing.assert_allclose(out[3:], [np.sqrt((Nv + Np) / Nf), np.sqrt(Nv / Nf)], rtol=1e-12)


def test_energy_norm_vanishes_at_the_discrete_solution():
    g, bx, by, _, _ = rand_problem(9, 8, 10)
    A, d = Dn.assemble(g)
    sol = np.linalg.solve(A, -d.pack(bx, by))
    vx, vy = d.unpack(sol)
    out = S.energy(g, vx, vy, bx, by)
    assert out[4] <= 1e-12


def test_energy_pressure_part_zero_for_divergence_free_mode():
    n = 32
    g = SimpleNamespace(nx=n, ny=n, dx=1 / n, dy=1 / n, eta_c=np.full((n, n), 2.0), eta_n=np.full((n + 1, n + 1), 2.0))
    xn, yc = np.arange(n + 1) / n, (np.arange(n) + 0.5) / n
    xc, yn = (np.arange(n) + 0.5) / n, np.arange(n + 1) / n
    vx = np.sin(np.pi * xn)[None, :] * np.cos(np.pi * yc)[:, None]
    vy = -np.cos(np.pi * xc)[None, :] * np.sin(np.pi * yn)[:, None]
    out = S.energy(g, vx, vy, np.ones((n, n + 1)), np.ones((n + 1, n)))
    assert out[1] <= 1e-26 * out[0]


# --------------------------------------------------- physical expectations --

def test_centred_sinker_mirror_symmetry():
    """The centred sinker is symmetric about x = 1/2: vx is odd, vy even
    (Sec. 6.1: the inclusion sinks vertically with a symmetric flow)."""
    p = I.centred_sinker(64)
    bx, by = S.rhs(p, p.fx, p.fy)
    vx, vy = p.zeros_v()
    for _ in range(20):
        vx, vy = S.jacobi(p, bx, by, 0.7, vx, vy)
    s = np.abs(vy).max()
    assert np.abs(vx + vx[:, ::-1]).max() <= 1e-12 * s
    assert np.abs(vy - vy[:, ::-1]).max() <= 1e-12 * s
    shifts = I.random_shifts(5, 64, 64, 1)
    rx, ry = S.smooth(p, *p.zeros_v(), p.fx, p.fy, None, 20, "ras", k=4, halo=4, tile_x=16, tile_y=16,
                      shifts=shifts)
    assert np.abs(rx - vx).max() <= 1e-13 * s and np.abs(ry - vy).max() <= 1e-13 * s


def test_sinker_sinks_with_two_vortices():
    """Solved flow: vy < 0 through the dense inclusion (gravity -y, Sec. 6.1),
    and vx changes sign across the inclusion (two counter-rotating cells)."""
    p = I.centred_sinker(32)
    levels = mg.hierarchy(p, coarsest=8)
    vx, vy, hist = mg.pcg(levels, p.fx, p.fy, tol=1e-9, max_iters=300)
    assert hist[-1] <= 1e-9
    assert vy[16, 15] < 0 and vy[16, 16] < 0
    assert vy[16, 15] == pytest.approx(vy.min(), rel=0.05)
    # above the sinker fluid moves inward-down on the left, right mirrored
    assert vx[24, 8] * vx[24, 24] < 0
