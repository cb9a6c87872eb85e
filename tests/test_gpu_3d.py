"""GPU 3D extension (the paper's future work) against the 3D oracle
(oracle/stokes3d.py), through the C ABI.

FP64: normwise max|GPU - oracle| / max|oracle| <= 1e-12 per component.
FP32: one sweep (one RAS outer iteration of k sweeps) from the same FP64
state rounded to FP32, <= 1e-5 (k * 1e-5).  RAS with an overlap >= k - 1 is k
Jacobi sweeps, so the GPU RAS must equal the GPU fused Jacobi bit for bit.
"""
import numpy as np
import pytest
import torch

from gpu_util import as_dtype, normwise
from oracle import stokes3d as S3
from paper_2509_19061_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_2509_19061_amd import api
    c = api.Context(0)
    yield c
    c.close()


def problem(nx, ny, nz, seed, contrast=1e4):
    rng = np.random.default_rng(seed)
    sph = [(float(a), float(b), float(c), float(r)) for a, b, c, r in
           zip(rng.uniform(0.2, 0.8, 4), rng.uniform(0.2, 0.8, 4), rng.uniform(0.2, 0.8, 4), rng.uniform(0.1, 0.25, 4))]
    return I.sinker_problem3d(nx, ny, nz, sph, contrast, 1.0)


def rounded(p, dtype):
    q = I.Problem3(p.nx, p.ny, p.nz, p.dx, p.dy, p.dz, *(as_dtype(a, dtype) for a in
                   (p.eta_c, p.eta_xy, p.eta_xz, p.eta_yz, p.fx, p.fy, p.fz)))
    return q


def gpu_run(ctx, p, dtype, v0, sweeps, variant, **opts):
    from paper_2509_19061_amd import api, fields
    dp = fields.DeviceProblem3(p, dtype)
    v = dp.velocity(v0)
    api.smooth3d(ctx, dtype, dp.grid, v, dp.eta, dp.f, sweeps, variant, **opts)
    torch.cuda.synchronize()
    return dp.get_v(v)


def oracle_jacobi(p, v, sweeps, omega=0.7):
    for _ in range(sweeps):
        v = S3.jacobi(p, p.fx, p.fy, p.fz, omega, *v)
    return v


@pytest.mark.parametrize("dims,sweeps", [((19, 14, 11), 3), ((8, 8, 8), 5), ((33, 9, 17), 2), ((130, 9, 40), 2)])
def test_jacobi3d_fp64_matches_oracle(ctx, dims, sweeps):
    p = problem(*dims, seed=sum(dims))
    v0 = I.random_velocity3d(p, 1, 1e-3)
    got = gpu_run(ctx, p, torch.float64, v0, sweeps, "jacobi_fused")
    ref = oracle_jacobi(p, v0, sweeps)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= TOL64


@pytest.mark.parametrize("T,h,k,sweeps", [(4, 0, 3, 6), (4, 1, 3, 5), (5, 2, 2, 4), (3, 0, 2, 2)])
def test_ras3d_matches_oracle(ctx, T, h, k, sweeps):
    """Thin and partial overlaps (a different smoother from Jacobi^k), explicit
    shifts, a partial last outer iteration, ragged tiles."""
    p = problem(17, 13, 11, 7 + T + h)
    v0 = I.random_velocity3d(p, 2, 1e-3)
    nout = (sweeps + k - 1) // k
    shifts = np.random.default_rng(T * 10 + h).integers(0, T, size=(nout, 3))
    got = gpu_run(ctx, p, torch.float64, v0, sweeps, "ras", tile=T, halo=h, k=k, shifts=shifts)
    v, left = v0, sweeps
    for t in range(nout):
        kt = min(k, left)
        v = S3.ras_outer(p, p.fx, p.fy, p.fz, 0.7, T, h, kt, tuple(shifts[t]), *v)
        left -= kt
    for g, r in zip(got, v):
        assert normwise(g, r) <= TOL64


@pytest.mark.parametrize("dims,T,k", [((40, 36, 30), 8, 2), ((64, 64, 64), 8, 2), ((50, 21, 33), 6, 3),
                                        ((130, 9, 40), 5, 2)])
def test_ras3d_full_overlap_equals_jacobi_bitwise(ctx, dims, T, k):
    """Overlap h = k: every outer iteration is k Jacobi sweeps exactly; the
    streaming tiles must reproduce the fused kernel bit for bit (random shifts)."""
    p = problem(*dims, seed=3)
    v0 = I.random_velocity3d(p, 4, 1e-3)
    a = gpu_run(ctx, p, torch.float64, v0, 2 * k, "ras", tile=T, halo=k, k=k, seed=5)
    b = gpu_run(ctx, p, torch.float64, v0, 2 * k, "jacobi_fused")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("variant,k", [("jacobi_fused", 1), ("ras", 2)])
def test_fp32_one_step_against_fp64_oracle(ctx, variant, k):
    p = problem(21, 16, 13, 9)
    p32 = rounded(p, torch.float32)
    v0 = tuple(as_dtype(a, torch.float32) for a in I.random_velocity3d(p, 6, 1e-3))
    kw = dict(tile=4, halo=0, k=k, shifts=np.array([[1, 2, 3]])) if variant == "ras" else {}
    got = gpu_run(ctx, p32, torch.float32, v0, k, variant, **kw)
    if variant == "ras":
        ref = S3.ras_outer(p32, p32.fx, p32.fy, p32.fz, 0.7, 4, 0, k, (1, 2, 3), *v0)
    else:
        ref = oracle_jacobi(p32, v0, 1)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= k * TOL32


def test_residual_and_energy3d_match_oracle(ctx):
    from paper_2509_19061_amd import api, fields
    p = problem(23, 17, 12, 11, contrast=1e5)
    v0 = I.random_velocity3d(p, 7, 1e-3)
    dp = fields.DeviceProblem3(p, torch.float64)
    v = dp.velocity(v0)
    r = dp.velocity()
    api.residual3d(ctx, torch.float64, dp.grid, v, dp.eta, dp.f, r)
    torch.cuda.synchronize()
    ref = S3.residual(p, *v0, p.fx, p.fy, p.fz)
    scale = max(np.abs(a).max() for a in ref)
    for g, o in zip(dp.get_v(r), ref):
        assert np.abs(g - o).max() <= TOL64 * scale
    e = api.energy_norm3d(ctx, torch.float64, dp.grid, v, dp.eta, dp.f)
    np.testing.assert_allclose(e, S3.energy(p, *v0, p.fx, p.fy, p.fz), rtol=1e-11)
    e2 = api.energy_norm3d(ctx, torch.float64, dp.grid, v, dp.eta, dp.f)
    assert np.array_equal(e, e2)
    # E_v = 1 at v = 0
    z = dp.velocity()
    assert api.energy_norm3d(ctx, torch.float64, dp.grid, z, dp.eta, dp.f)[2] == pytest.approx(1.0, abs=1e-14)


def test_3d_errors(ctx):
    from paper_2509_19061_amd import api, fields
    p = problem(8, 8, 8, 12)
    dp = fields.DeviceProblem3(p, torch.float64)
    v = dp.velocity()
    with pytest.raises(api.StkError) as e:  # 6 (64 + 2 + 2)^3 doubles do not fit in LDS
        api.smooth3d(ctx, torch.float64, dp.grid, v, dp.eta, dp.f, 2, "ras", tile=64, k=1)
    assert e.value.code == api.EUNSUPPORTED
    with pytest.raises(api.StkError) as e:
        api.smooth3d(ctx, torch.float64, dp.grid, v, dp.eta, dp.f, 2, "rbgs")
    assert e.value.code == api.EINVAL
