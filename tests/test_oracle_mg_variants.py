"""Pins of the oracle's smoother variants inside the V-cycle (Sec. 6.2, 6.3):
RAS-type temporal blocking (Alg. 2) on a level's assembled operator, the
mixed smoother and the per-level sweep schedule.

* one tile covering the level is k Jacobi sweeps (bitwise: the same rows);
* with an overlap at least the stencil reach times (k - 1) an outer
  iteration is k Jacobi sweeps for any tile size and shift (every value a row
  reads lies inside its tile's region for the sweeps that matter): reach 1 on
  the finest level, 2 on the Galerkin levels;
* the same tile update written with dense blocks (frozen ring moved to the
  right-hand side) on small grids;
* a thin overlap is a different smoother (differs from Jacobi^k);
* the general V-cycle with no variant is the plain V-cycle bit for bit, and a
  coarse RAS with enough overlap leaves it unchanged;
* a relaxed coarsest level with many sweeps reaches the exact coarse solve;
* the sweep schedule nu * 2.5^l: 5, 13, 31, 78.
"""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import mg
from oracle import sparse as SP
from paper_2509_19061_amd import inputs as I


def _problem(nx, ny, seed, contrast):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.2, 0.8, size=(3, 2))
    r = rng.uniform(0.06, 0.12, size=3)
    return I.sinker_problem(nx, ny, [(float(c[k, 0]), float(c[k, 1]), float(r[k])) for k in range(3)], contrast, 1.0)


def _jacobi(L, x, c, k, omega):
    for _ in range(k):
        x = x + omega * (c - L.A @ x) / L.D
    return x


def _rand(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


@pytest.mark.parametrize("lev", [0, 1, 2])
def test_one_tile_is_jacobi(lev):
    levels = mg.hierarchy(_problem(48, 40, 3, 1e3))
    L = levels[lev]
    n = L.A.shape[0]
    x, c = _rand(n, 1), _rand(n, 2)
    got = mg.ras_level(L, x, c, T=64, h=0, k=3, omega=0.7)
    assert np.array_equal(got, _jacobi(L, x, c, 3, 0.7))


@pytest.mark.parametrize("lev,reach", [(0, 1), (1, 2), (2, 2)])
@pytest.mark.parametrize("T,k,shift", [(8, 2, (0, 0)), (7, 3, (3, 5)), (5, 4, (4, 1))])
def test_overlap_of_reach_times_k_minus_1_is_jacobi(lev, reach, T, k, shift):
    levels = mg.hierarchy(_problem(48, 40, 5, 1e4))
    L = levels[lev]
    n = L.A.shape[0]
    x, c = _rand(n, 3), _rand(n, 4)
    got = mg.ras_level(L, x, c, T=T, h=reach * (k - 1), k=k, omega=0.6, shift=shift)
    assert np.array_equal(got, _jacobi(L, x, c, k, 0.6))


def test_thin_overlap_differs_from_jacobi():
    L = mg.hierarchy(_problem(48, 40, 6, 1e4))[1]
    n = L.A.shape[0]
    x, c = _rand(n, 5), _rand(n, 6)
    got = mg.ras_level(L, x, c, T=6, h=0, k=4, omega=0.7, shift=(2, 1))
    ref = _jacobi(L, x, c, 4, 0.7)
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()
    # a halo one short of the reach-times-(k-1) bound also differs
    got = mg.ras_level(L, x, c, T=6, h=2 * 3 - 1, k=4, omega=0.7, shift=(2, 1))
    assert np.abs(got - ref).max() > 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("h,k,shift", [(0, 3, (1, 2)), (1, 2, (0, 0)), (2, 4, (3, 3))])
def test_tile_update_matches_dense_block_form(h, k, shift):
    """Each tile: z_E <- z_E + omega D_E^-1 (c_E - A_EE z_E - A_ER u_R), with
    A_ER the couplings to every unknown outside E (held at the snapshot u),
    from dense blocks; owned unknowns kept."""
    L = mg.hierarchy(_problem(16, 12, 7, 1e3))[1]  # 8 x 6 coarse cells
    A = L.A.toarray()
    n = A.shape[0]
    x, c = _rand(n, 7), _rand(n, 8)
    T = 3
    nvx, vx_id, vy_id = SP.numbering(L.nx, L.ny)
    out = x.copy()
    for (x0, x1) in mg.tile_intervals(L.nx, T, shift[0]):
        for (y0, y1) in mg.tile_intervals(L.ny, T, shift[1]):
            inE = np.zeros(n, bool)
            own = np.zeros(n, bool)
            for j in range(L.ny + 1):
                for i in range(L.nx + 1):
                    inside = max(x0 - h, 0) <= i < min(x1 + h, L.nx) and max(y0 - h, 0) <= j < min(y1 + h, L.ny)
                    owned = x0 <= i < x1 and y0 <= j < y1
                    for ids in (vx_id, vy_id):
                        if j < ids.shape[0] and i < ids.shape[1] and ids[j, i] >= 0:
                            inE[ids[j, i]] |= inside
                            own[ids[j, i]] |= owned
            E, R = np.flatnonzero(inE), np.flatnonzero(~inE)
            rhs = c[E] - A[np.ix_(E, R)] @ x[R]
            z = x[E].copy()
            for _ in range(k):
                z = z + 0.7 * (rhs - A[np.ix_(E, E)] @ z) / np.diag(A)[E]
            full = x.copy()
            full[E] = z
            out[own] = full[own]
    got = mg.ras_level(L, x, c, T=T, h=h, k=k, omega=0.7, shift=shift)
    assert np.abs(got - out).max() <= 1e-13 * np.abs(out).max()


def test_general_vcycle_defaults_are_the_plain_vcycle_and_safe_coarse_ras_changes_nothing():
    p = _problem(64, 48, 8, 1e3)
    levels = mg.hierarchy(p)
    n = levels[0].A.shape[0]
    x, c = _rand(n, 9), _rand(n, 10)
    ref = mg._vcycle_packed(levels, 0, x, c, 2, 2, 0.7)
    assert np.array_equal(mg.vcycle_general(levels, 0, x, c), ref)
    # coarse RAS with overlap 2 (k - 1) on the Galerkin levels: Jacobi there, so the same cycle
    got = mg.vcycle_general(levels, 0, x, c, coarse=dict(T=8, h=2, k=2))
    assert np.array_equal(got, ref)
    # the mixed smoother with the paper's thin overlap is a different cycle
    got = mg.vcycle_general(levels, 0, x, c, coarse=dict(T=8, h=0, k=2))
    assert np.abs(got - ref).max() > 1e-6 * np.abs(ref).max()
    # so is a finest-level RAS with halo 0
    got = mg.vcycle_general(levels, 0, x, c, fine=dict(T=16, h=0, k=2))
    assert np.abs(got - ref).max() > 1e-6 * np.abs(ref).max()


def test_relaxed_coarsest_level_reaches_the_exact_coarse_solve():
    p = _problem(16, 16, 9, 1e2)
    levels = mg.hierarchy_truncated(p, 2)  # 16^2 and 8^2
    assert len(levels) == 2
    n = levels[0].A.shape[0]
    x, c = _rand(n, 11), _rand(n, 12)
    exact = mg.vcycle_general(levels, 0, x, c)
    # 2 + 2 sweeps on the coarse level do not solve it; 4000 + 4000 do
    far = mg.vcycle_general(levels, 0, x, c, relax_coarsest=True)
    assert np.abs(far - exact).max() > 1e-2 * np.abs(exact).max()
    relaxed = mg.vcycle_general(levels, 0, x, c, growth=2000.0, relax_coarsest=True)
    assert np.abs(relaxed - exact).max() <= 1e-12 * np.abs(exact).max()


def test_sweep_schedule():
    assert [mg.sweeps_per_level(5, 2.5, l) for l in range(4)] == [5, 13, 31, 78]
    assert [mg.sweeps_per_level(2, 1.0, l) for l in range(5)] == [2] * 5
    assert mg.tile_intervals(10, 4, 0) == [(0, 4), (4, 8), (8, 10)]
    assert mg.tile_intervals(10, 4, 3) == [(0, 3), (3, 7), (7, 10)]
    assert mg.tile_intervals(10, 4, 6) == [(0, 2), (2, 6), (6, 10)]
