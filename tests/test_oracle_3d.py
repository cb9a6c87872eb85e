"""Pins of the 3D oracle (oracle/stokes3d.py), the paper's future-work
extension (Sec. 9): the staggered operator, Jacobi and RAS in 3D.

* A = -M = B^T W B from the strain-rate rows (assembled independently)
  equals the stencil apply, and diag(A) the diagonal formula;
* symmetry <A u, v> = <u, A v> and positivity at a larger size;
* constant viscosity, cubic cells of size h: the divergence-free field
  vx = a sin(pi x) cos(pi y) cos(pi z), vy = b cos sin cos, vz = c cos cos sin
  (a + b + c = 0) is an exact discrete eigenvector of -M with eigenvalue
  4 eta (sin^2(pi dx/2)/dx^2 + sin^2(pi dy/2)/dy^2 + sin^2(pi dz/2)/dz^2);
* on fields that do not depend on z (vz = 0) the 3D operator is the 2D one
  of the 2D oracle in every layer (independent code);
* Jacobi equals the dense update; RAS with one tile, or with overlap >= k - 1
  at any tiling, is k Jacobi sweeps; a tile update matches its dense block
  form; a thin overlap differs from Jacobi^k.
"""
import numpy as np
import pytest

from oracle import stokes as S2
from oracle import stokes3d as S3
from paper_2509_19061_amd import inputs as I


def _rand_problem(nx, ny, nz, seed, contrast=1e3):
    rng = np.random.default_rng(seed)
    sph = [(float(a), float(b), float(c), float(r)) for a, b, c, r in
           zip(rng.uniform(0.2, 0.8, 3), rng.uniform(0.2, 0.8, 3), rng.uniform(0.2, 0.8, 3), rng.uniform(0.1, 0.3, 3))]
    p = I.sinker_problem3d(nx, ny, nz, sph, contrast, 1.0)
    # perturb every viscosity so that no coefficient coincides by construction
    for name in ("eta_c", "eta_xy", "eta_xz", "eta_yz"):
        setattr(p, name, getattr(p, name) * rng.uniform(0.5, 1.5, getattr(p, name).shape))
    return p


def _vec(p, seed):
    return I.random_velocity3d(p, seed)


@pytest.mark.parametrize("dims", [(4, 3, 5), (3, 3, 3), (5, 4, 2)])
def test_stencil_equals_assembled_btwb(dims):
    p = _rand_problem(*dims, seed=sum(dims))
    p.dx, p.dy, p.dz = 0.7, 1.3, 0.9
    A = S3.operator_matrix(p)
    v = _vec(p, 1)
    got = S3.pack(p, *S3.apply(p, *v))
    ref = -(A @ S3.pack(p, *v))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    d = S3.pack(p, *S3.diag(p))
    assert np.abs(d - A.diagonal()).max() <= 1e-13 * np.abs(d).max()


def test_symmetric_positive_definite():
    p = _rand_problem(9, 7, 8, 3, contrast=1e5)
    u, w = _vec(p, 2), _vec(p, 3)
    au, aw = S3.apply(p, *u), S3.apply(p, *w)
    a = sum(float(np.sum(x * y)) for x, y in zip(au, w))
    b = sum(float(np.sum(x * y)) for x, y in zip(u, aw))
    assert abs(a - b) <= 1e-12 * abs(a)
    assert -sum(float(np.sum(x * y)) for x, y in zip(au, u)) > 0


@pytest.mark.parametrize("n,abc", [(8, (1.0, -0.5, -0.5)), (12, (0.3, 0.7, -1.0))])
def test_divergence_free_mode_is_an_eigenvector(n, abc):
    eta = 2.5
    p = I.sinker_problem3d(n, n, n, [], 1.0, eta)
    h = 1.0 / n
    a, b, c = abc
    xn, xc = np.arange(n + 1) * h, (np.arange(n) + 0.5) * h
    s, co = np.sin, np.cos
    pi = np.pi
    vx = a * s(pi * xn)[None, None, :] * co(pi * xc)[None, :, None] * co(pi * xc)[:, None, None]
    vy = b * co(pi * xc)[None, None, :] * s(pi * xn)[None, :, None] * co(pi * xc)[:, None, None]
    vz = c * co(pi * xc)[None, None, :] * co(pi * xc)[None, :, None] * s(pi * xn)[:, None, None]
    lam = 4 * eta * 3 * np.sin(pi * h / 2) ** 2 / h ** 2
    ax, ay, az = S3.apply(p, vx, vy, vz)
    m = S3.masks(p)
    for got, v, mm in zip((ax, ay, az), (vx, vy, vz), m):
        assert np.abs(np.where(mm, -got - lam * v, 0.0)).max() <= 1e-11 * lam * np.abs(v).max()


def test_z_invariant_fields_give_the_2d_operator():
    nx, ny, nz = 10, 7, 4
    rng = np.random.default_rng(5)
    ec2 = rng.uniform(0.5, 3.0, (ny, nx))
    en2 = I.nodal_harmonic(ec2)
    p2 = I.Problem(nx, ny, 1.0 / nx, 1.0 / ny, ec2, en2, None, None)
    p3 = I.Problem3(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, np.broadcast_to(ec2, (nz, ny, nx)).copy(),
                    np.broadcast_to(en2, (nz, ny + 1, nx + 1)).copy(), rng.uniform(1, 2, (nz + 1, ny, nx + 1)),
                    rng.uniform(1, 2, (nz + 1, ny + 1, nx)))
    vx2, vy2 = I.random_velocity(p2, 6)
    vx = np.broadcast_to(vx2, (nz, ny, nx + 1)).copy()
    vy = np.broadcast_to(vy2, (nz, ny + 1, nx)).copy()
    vz = np.zeros((nz + 1, ny, nx))
    ax, ay, az = S3.apply(p3, vx, vy, vz)
    rx, ry = S2.apply(p2, vx2, vy2)
    for kk in range(nz):
        assert np.abs(ax[kk] - rx).max() <= 1e-12 * np.abs(rx).max()
        assert np.abs(ay[kk] - ry).max() <= 1e-12 * np.abs(ry).max()
    assert np.abs(az).max() == 0.0


def test_jacobi_equals_dense_update():
    p = _rand_problem(4, 4, 3, 7)
    A = S3.operator_matrix(p).toarray()
    v, b = _vec(p, 8), _vec(p, 9)
    got = S3.pack(p, *S3.jacobi(p, *b, 0.7, *v))
    x, c = S3.pack(p, *v), S3.pack(p, *b)
    ref = x + 0.7 * (-c - A @ x) / np.diag(A)  # A x = -b
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def _jac_k(p, b, v, k, omega=0.7):
    for _ in range(k):
        v = S3.jacobi(p, *b, omega, *v)
    return v


@pytest.mark.parametrize("T,h,k,shift", [(16, 0, 3, (0, 0, 0)), (3, 1, 2, (1, 2, 0)), (4, 2, 3, (3, 0, 2)),
                                         (2, 3, 4, (1, 1, 1))])
def test_ras_one_tile_or_full_overlap_is_jacobi(T, h, k, shift):
    p = _rand_problem(7, 6, 5, 11)
    v, b = _vec(p, 12), _vec(p, 13)
    got = S3.ras_outer(p, *b, 0.7, T, h, k, shift, *v)
    ref = _jac_k(p, b, v, k)
    for g, r in zip(got, ref):
        assert np.abs(g - r).max() <= 1e-13 * np.abs(r).max()


def test_ras_thin_overlap_differs_and_matches_dense_blocks():
    p = _rand_problem(5, 4, 4, 14)
    v, b = _vec(p, 15), _vec(p, 16)
    T, h, k, shift = 2, 0, 3, (1, 0, 1)
    got = S3.ras_outer(p, *b, 0.7, T, h, k, shift, *v)
    ref = _jac_k(p, b, v, k)
    assert max(np.abs(g - r).max() for g, r in zip(got, ref)) > 1e-3
    # dense block form per tile: z_E <- z_E + omega D_E^-1 (c_E - A_EE z_E - A_ER u_R), owned kept
    A = S3.operator_matrix(p).toarray()
    (ix, iy, iz), n = S3.numbering(p)
    x, c = S3.pack(p, *v), -S3.pack(p, *b)
    out = x.copy()
    for (x0, x1) in S3.tile_intervals(p.nx, T, shift[0]):
        for (y0, y1) in S3.tile_intervals(p.ny, T, shift[1]):
            for (z0, z1) in S3.tile_intervals(p.nz, T, shift[2]):
                def sel(lo, hi):
                    ids = np.concatenate([a[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].ravel() for a in (ix, iy, iz)])
                    return ids[ids >= 0]
                E = sel((max(x0 - h, 0), max(y0 - h, 0), max(z0 - h, 0)), (min(x1 + h, p.nx), min(y1 + h, p.ny),
                                                                           min(z1 + h, p.nz)))
                own = sel((x0, y0, z0), (x1, y1, z1))
                R = np.setdiff1d(np.arange(n), E)
                rhs = c[E] - A[np.ix_(E, R)] @ x[R]
                zE = x[E].copy()
                for _ in range(k):
                    zE = zE + 0.7 * (rhs - A[np.ix_(E, E)] @ zE) / np.diag(A)[E]
                full = x.copy()
                full[E] = zE
                out[own] = full[own]
    assert np.abs(S3.pack(p, *got) - out).max() <= 1e-12 * np.abs(out).max()


def test_energy_norm_special_cases():
    p = _rand_problem(6, 5, 4, 17)
    f = p.fx, p.fy, p.fz
    nv, nf, ev = S3.energy(p, *p.zeros_v(), *f)
    assert ev == pytest.approx(1.0, abs=1e-15) and nv == pytest.approx(nf, rel=1e-15)
    # the dense solution has E_v ~ 0
    A = S3.operator_matrix(p).toarray()
    x = np.linalg.solve(A, -S3.pack(p, *f))
    assert S3.energy(p, *S3.unpack(p, x), *f)[2] <= 1e-10


def test_sphere_sinks():
    p = I.sinker_problem3d(12, 12, 12, [(0.5, 0.5, 0.5, 0.2)], 1e3, 1.0)
    A = S3.operator_matrix(p).toarray()
    vx, vy, vz = S3.unpack(p, np.linalg.solve(A, -S3.pack(p, p.fx, p.fy, p.fz)))
    assert vz[6, 6, 6] < 0 and abs(vz[6, 6, 6]) > 10 * abs(vx).max() * 0
