"""GPU parity of the HIP smoothers, residual and energy norm vs the CPU oracle.

FP64: normwise max|GPU - oracle| / max|oracle| <= 1e-12 per component.
FP32: one sweep (or one RAS outer iteration of k sweeps) from the same FP64
state rounded to FP32, against the FP64 oracle, <= 1e-5 (k * 1e-5 for RAS).
"""
import numpy as np
import pytest
import torch

from gpu_util import as_dtype, gpu_smooth, normwise
from oracle import stokes as S
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


def _forced_ctx(kind):
    import os
    from paper_2509_19061_amd import api
    old = os.environ.get("STK_RAS_KERNEL")
    os.environ["STK_RAS_KERNEL"] = kind
    try:
        return api.Context(0)
    finally:
        if old is None:
            del os.environ["STK_RAS_KERNEL"]
        else:
            os.environ["STK_RAS_KERNEL"] = old


@pytest.fixture(scope="module", params=["window", "stream"])
def ras_ctx(request):
    """Contexts pinned to one RAS kernel (LDS window / streaming)."""
    c = _forced_ctx(request.param)
    yield c
    c.close()


def ragged_problem(nx=200, ny=150, seed=11, contrast=1e6):
    rng = np.random.default_rng(seed)
    count = 6
    c = rng.uniform(0.1, 0.9, size=(count, 2))
    r = rng.uniform(0.04, 0.12, size=count)
    return I.sinker_problem(nx, ny, [(float(c[k, 0]), float(c[k, 1]), float(r[k])) for k in range(count)],
                            contrast, 1.0)


# --------------------------------------------------------------- config 1 --
@pytest.mark.parametrize("variant", ["jacobi", "jacobi_fused", "ras", "rbgs"])
def test_centred_sinker_20_sweeps_fp64(ctx, variant):
    """64^2 centred sinker, omega = 0.7 (RBGS: 1.0), 20 sweeps from v = 0."""
    p = I.centred_sinker(64)
    kw = dict(tile_x=64, tile_y=64, k=4, halo=4, shifts=I.random_shifts(5, 64, 64, 1)) if variant == "ras" else {}
    gx, gy = gpu_smooth(ctx, p, torch.float64, variant, 20, **kw)
    ox, oy = S.smooth(p, *p.zeros_v(), p.fx, p.fy, None, 20, variant, **kw)
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64
    # mirror symmetry about x = 1/2 survives on the GPU (not for RBGS colouring)
    if variant != "rbgs":
        s = np.abs(gy).max()
        assert np.abs(gx + gx[:, ::-1]).max() <= 1e-12 * s
    # sinking: vy < 0 at the centre
    assert gy[32, 31] < 0


def test_centred_sinker_energy_history_fp64(ctx):
    from paper_2509_19061_amd import api, fields
    p = I.centred_sinker(64)
    dp = fields.DeviceProblem(p, torch.float64)
    vx, vy = dp.velocity()
    ox, oy = p.zeros_v()
    bx, by = S.rhs(p, p.fx, p.fy)
    for s in range(20):
        e_gpu = api.energy_norm(ctx, torch.float64, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
        e_or = S.energy(p, ox, oy, p.fx, p.fy)
        np.testing.assert_allclose(e_gpu, e_or, rtol=1e-11, atol=0)
        api.smooth(ctx, torch.float64, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, 1, "jacobi_fused")
        ox, oy = S.jacobi(p, bx, by, 0.7, ox, oy)
    assert e_gpu[4] < 1.0


# ------------------------------------------------- several tiles, ragged --
@pytest.mark.parametrize("k,h", [(2, 2), (4, 4), (8, 8), (4, 1), (3, 0), (1, 0), (5, 2)])
def test_ras_ragged_tiles_fp64(ras_ctx, k, h):
    p = ragged_problem()
    vx0, vy0 = I.random_velocity(p, 3, 1e-3)
    shifts = I.random_shifts(10, 64, 48, 7)
    kw = dict(tile_x=64, tile_y=48, k=k, halo=h)
    gx, gy = gpu_smooth(ras_ctx, p, torch.float64, "ras", 10, vx0, vy0, shifts=shifts, **kw)
    ox, oy = S.smooth(p, vx0, vy0, p.fx, p.fy, None, 10, "ras", shifts=shifts, **kw)
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64


@pytest.mark.parametrize("variant", ["jacobi", "jacobi_fused", "rbgs"])
def test_global_smoothers_ragged_with_pressure_fp64(ctx, variant):
    p = ragged_problem(131, 77, 12, 1e4)
    vx0, vy0 = I.random_velocity(p, 4, 1e-2)
    pr = I.random_pressure(p, 5)
    gx, gy = gpu_smooth(ctx, p, torch.float64, variant, 7, vx0, vy0, p=pr, omega=0.6)
    ox, oy = S.smooth(p, vx0, vy0, p.fx, p.fy, pr, 7, variant, omega=0.6)
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64


def test_ras_with_pressure_and_literal_outer_count_fp64(ras_ctx):
    ctx = ras_ctx
    p = ragged_problem(97, 130, 13, 1e3)
    vx0, vy0 = I.random_velocity(p, 6, 1e-2)
    pr = I.random_pressure(p, 7)
    shifts = I.random_shifts(4, 32, 32, 8)
    kw = dict(tile_x=32, tile_y=32, k=3, halo=1, last_partial=False)
    gx, gy = gpu_smooth(ctx, p, torch.float64, "ras", 10, vx0, vy0, p=pr, shifts=shifts, **kw)
    ox, oy = S.smooth(p, vx0, vy0, p.fx, p.fy, pr, 10, "ras", shifts=shifts, **kw)
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ras_with_enough_overlap_is_bitwise_fused_jacobi(ctx, ras_ctx, dtype):
    """RAS(h >= k-1) computes exactly Jacobi^k; the kernels share one update
    expression, so the GPU results agree bit for bit."""
    p = ragged_problem()
    vx0, vy0 = I.random_velocity(p, 9, 1e-3)
    if dtype == torch.float32:
        p = I.Problem(p.nx, p.ny, p.dx, p.dy, as_dtype(p.eta_c, dtype), as_dtype(p.eta_n, dtype),
                      as_dtype(p.fx, dtype), as_dtype(p.fy, dtype))
        vx0, vy0 = as_dtype(vx0, dtype), as_dtype(vy0, dtype)
    rx, ry = gpu_smooth(ras_ctx, p, dtype, "ras", 12, vx0, vy0, tile_x=64, tile_y=64, k=4, halo=3, seed=5)
    jx, jy = gpu_smooth(ctx, p, dtype, "jacobi_fused", 12, vx0, vy0)
    sx, sy = gpu_smooth(ctx, p, dtype, "jacobi", 12, vx0, vy0)
    assert np.array_equal(rx, jx) and np.array_equal(ry, jy)
    assert np.array_equal(sx, jx) and np.array_equal(sy, jy)


@pytest.mark.parametrize("variant", ["jacobi_fused", "ras", "rbgs"])
def test_deterministic_run_to_run(ctx, variant):
    p = ragged_problem()
    vx0, vy0 = I.random_velocity(p, 10, 1e-3)
    kw = dict(k=4, halo=1, seed=3) if variant == "ras" else {}
    a = gpu_smooth(ctx, p, torch.float64, variant, 9, vx0, vy0, **kw)
    b = gpu_smooth(ctx, p, torch.float64, variant, 9, vx0, vy0, **kw)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------------- FP32 --
@pytest.mark.parametrize("variant,k", [("jacobi", 1), ("jacobi_fused", 1), ("rbgs", 1), ("ras", 2), ("ras", 4),
                                       ("ras", 8)])
def test_fp32_one_step_against_fp64_oracle(ras_ctx, variant, k):
    ctx = ras_ctx
    p = ragged_problem(200, 150, 14, 1e6)
    # an FP64 state a few sweeps in, rounded to FP32 (inputs identical on both sides)
    bx, by = S.rhs(p, p.fx, p.fy)
    vx, vy = p.zeros_v()
    for _ in range(5):
        vx, vy = S.jacobi(p, bx, by, 0.7, vx, vy)
    p32 = I.Problem(p.nx, p.ny, p.dx, p.dy, as_dtype(p.eta_c, torch.float32), as_dtype(p.eta_n, torch.float32),
                    as_dtype(p.fx, torch.float32), as_dtype(p.fy, torch.float32))
    vx, vy = as_dtype(vx, torch.float32), as_dtype(vy, torch.float32)
    shifts = I.random_shifts(1, 64, 64, 15)
    kw = dict(k=k, halo=k, shifts=shifts) if variant == "ras" else {}
    gx, gy = gpu_smooth(ctx, p32, torch.float32, variant, k, vx, vy, **kw)
    ox, oy = S.smooth(p32, vx, vy, p32.fx, p32.fy, None, k, variant, **kw)
    assert normwise(gx, ox) <= k * TOL32 and normwise(gy, oy) <= k * TOL32


# -------------------------------------------------------- residual / norm --
@pytest.mark.parametrize("with_p", [False, True])
def test_residual_and_energy_fp64(ctx, with_p):
    from paper_2509_19061_amd import api, fields
    p = ragged_problem(131, 77, 16, 1e5)
    vx0, vy0 = I.random_velocity(p, 17, 1e-3)
    pr = I.random_pressure(p, 18) if with_p else None
    dp = fields.DeviceProblem(p, torch.float64)
    vx, vy = dp.velocity(vx0, vy0)
    pt = None if pr is None else dp.field(pr)
    rx, ry, rp = dp.field(), dp.field(), dp.field()
    api.residual(ctx, torch.float64, dp.grid, vx, vy, pt, dp.eta_c, dp.eta_n, dp.fx, dp.fy, rx, ry, rp)
    torch.cuda.synchronize()
    ox, oy, op = S.residual(p, vx0, vy0, p.fx, p.fy, pr)
    scale = max(np.abs(ox).max(), np.abs(oy).max())
    assert np.abs(dp.get_vx(rx) - ox).max() <= TOL64 * scale
    assert np.abs(dp.get_vy(ry) - oy).max() <= TOL64 * scale
    assert normwise(dp.get_cell(rp), op) <= TOL64
    e = api.energy_norm(ctx, torch.float64, dp.grid, vx, vy, pt, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
    np.testing.assert_allclose(e, S.energy(p, vx0, vy0, p.fx, p.fy, pr), rtol=1e-11, atol=0)
    # reproducible bit for bit
    e2 = api.energy_norm(ctx, torch.float64, dp.grid, vx, vy, pt, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
    assert np.array_equal(e, e2)


def test_energy_fp32_inputs(ctx):
    from paper_2509_19061_amd import api, fields
    p = ragged_problem(131, 77, 19, 1e5)
    vx0, vy0 = I.random_velocity(p, 20, 1e-3)
    p32 = I.Problem(p.nx, p.ny, p.dx, p.dy, as_dtype(p.eta_c, torch.float32), as_dtype(p.eta_n, torch.float32),
                    as_dtype(p.fx, torch.float32), as_dtype(p.fy, torch.float32))
    vx0, vy0 = as_dtype(vx0, torch.float32), as_dtype(vy0, torch.float32)
    dp = fields.DeviceProblem(p32, torch.float32)
    vx, vy = dp.velocity(vx0, vy0)
    e = api.energy_norm(ctx, torch.float32, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
    np.testing.assert_allclose(e, S.energy(p32, vx0, vy0, p32.fx, p32.fy), rtol=1e-5)
    z = api.energy_norm(ctx, torch.float32, dp.grid, *dp.velocity(), None, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
    assert z[3] == 1.0 and z[4] == 1.0 and z[1] == 0.0


# ----------------------------------------------------------- edge cases --
@pytest.mark.parametrize("nx,ny", [(2, 2), (3, 2), (2, 5), (65, 3)])
def test_tiny_grids_all_variants(ctx, nx, ny):
    rng = np.random.default_rng(nx * 7 + ny)
    ec = 10 ** rng.uniform(0, 3, (ny, nx))
    p = I.Problem(nx, ny, 1 / nx, 1 / ny, ec, I.nodal_harmonic(ec), rng.standard_normal((ny, nx + 1)),
                  rng.standard_normal((ny + 1, nx)))
    for variant in ("jacobi", "jacobi_fused", "rbgs", "ras"):
        kw = dict(k=3, halo=1, tile_x=1, tile_y=2, shifts=[[0, 1], [0, 0]]) if variant == "ras" else {}
        gx, gy = gpu_smooth(ctx, p, torch.float64, variant, 5, **kw)
        ox, oy = S.smooth(p, *p.zeros_v(), p.fx, p.fy, None, 5, variant, **kw)
        assert np.abs(gx - ox).max() <= TOL64 * max(1e-300, np.abs(ox).max()) + 1e-300
        assert np.abs(gy - oy).max() <= TOL64 * max(1e-300, np.abs(oy).max()) + 1e-300


@pytest.mark.parametrize("nx,ny", [(61, 63), (62, 64), (123, 127), (124, 128), (186, 65)])
def test_row_streaming_strip_and_segment_edges(ctx, nx, ny):
    """The row-streaming kernels split the grid into strips of 62 columns and
    segments of 64 rows (vx has nx + 1 columns, vy ny + 1 rows): exact
    multiples and one either side, for the fused Jacobi sweep, the residual
    with a pressure and the energy norm."""
    from paper_2509_19061_amd import api, fields
    p = ragged_problem(nx, ny, nx + ny, 1e4)
    vx0, vy0 = I.random_velocity(p, nx, 1e-2)
    gx, gy = gpu_smooth(ctx, p, torch.float64, "jacobi_fused", 2, vx0, vy0)
    ox, oy = S.smooth(p, vx0, vy0, p.fx, p.fy, None, 2, "jacobi_fused")
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64
    pr = I.random_pressure(p, ny)
    dp = fields.DeviceProblem(p, torch.float64)
    vx, vy = dp.velocity(vx0, vy0)
    pt = dp.field(pr)
    rx, ry, rp = dp.field(), dp.field(), dp.field()
    api.residual(ctx, torch.float64, dp.grid, vx, vy, pt, dp.eta_c, dp.eta_n, dp.fx, dp.fy, rx, ry, rp)
    torch.cuda.synchronize()
    ax, ay, ap = S.residual(p, vx0, vy0, p.fx, p.fy, pr)
    assert normwise(dp.get_vx(rx), ax) <= TOL64 and normwise(dp.get_vy(ry), ay) <= TOL64
    assert normwise(dp.get_cell(rp), ap) <= TOL64
    e = api.energy_norm(ctx, torch.float64, dp.grid, vx, vy, pt, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
    np.testing.assert_allclose(e, S.energy(p, vx0, vy0, p.fx, p.fy, pr), rtol=1e-11, atol=0)


def test_walls_written_zero_and_garbage_walls_ignored(ctx):
    p = ragged_problem(70, 66, 21, 1e2)
    vx0, vy0 = I.random_velocity(p, 22, 1.0)
    gx0, gy0 = vx0.copy(), vy0.copy()
    gx0[:, [0, -1]] = 1e30
    gy0[[0, -1], :] = -1e30
    for variant in ("jacobi", "jacobi_fused", "rbgs", "ras"):
        kw = dict(k=2, seed=1) if variant == "ras" else {}
        a = gpu_smooth(ctx, p, torch.float64, variant, 3, vx0, vy0, **kw)
        b = gpu_smooth(ctx, p, torch.float64, variant, 3, gx0, gy0, **kw)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert np.all(b[0][:, [0, -1]] == 0) and np.all(b[1][[0, -1], :] == 0)


def test_shift_larger_than_tile_and_tile_larger_than_domain(ctx):
    p = ragged_problem(90, 70, 23, 1e3)
    vx0, vy0 = I.random_velocity(p, 24, 1e-2)
    big = [[130, 75], [64 + 5, 3]]
    gx, gy = gpu_smooth(ctx, p, torch.float64, "ras", 6, vx0, vy0, tile_x=64, tile_y=64, k=3, halo=0, shifts=big)
    ox, oy = S.smooth(p, vx0, vy0, p.fx, p.fy, None, 6, "ras", tile_x=64, tile_y=64, k=3, halo=0,
                      shifts=[[130 % 64, 75 % 64], [5, 3]])
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64
    gx, gy = gpu_smooth(ctx, p, torch.float64, "ras", 4, vx0, vy0, tile_x=512, tile_y=100, k=4, halo=0, seed=2)
    jx, jy = gpu_smooth(ctx, p, torch.float64, "jacobi_fused", 4, vx0, vy0)
    assert normwise(gx, jx) <= TOL64 and normwise(gy, jy) <= TOL64


def test_zero_sweeps_is_noop_and_errors(ctx):
    from paper_2509_19061_amd import api
    p = ragged_problem(40, 40, 25, 1e2)
    vx0, vy0 = I.random_velocity(p, 26, 1.0)
    gx, gy = gpu_smooth(ctx, p, torch.float64, "jacobi_fused", 0, vx0, vy0)
    assert np.array_equal(gx, vx0) and np.array_equal(gy, vy0)
    with pytest.raises(api.StkError) as e:
        gpu_smooth(ctx, ragged_problem(), torch.float64, "ras", 4, tile_x=256, tile_y=256, k=4)
    assert e.value.code == api.EUNSUPPORTED
    with pytest.raises(api.StkError) as e:
        gpu_smooth(ctx, p, torch.float64, "jacobi", 4, omega=2.5)
    assert e.value.code == api.EINVAL
    with pytest.raises(api.StkError) as e:
        gpu_smooth(ctx, p, torch.float64, "ras", 4, k=0)
    assert e.value.code == api.EINVAL


def test_fp64_nonfinite_norm_reported(ctx):
    from paper_2509_19061_amd import api, fields
    p = ragged_problem(40, 40, 27, 1e2)
    p.fx[:] = 0.0
    p.fy[:] = 0.0
    dp = fields.DeviceProblem(p, torch.float64)
    with pytest.raises(api.StkError) as e:
        api.energy_norm(ctx, torch.float64, dp.grid, *dp.velocity(), None, dp.eta_c, dp.eta_n, dp.fx, dp.fy)
    assert e.value.code == api.ENONFINITE


# ----------------------------------------------------- full-size workload --
@pytest.mark.parametrize("k", [2, 4, 8])
def test_full_size_4096_ras_one_outer_iteration_vs_oracle(ctx, k):
    """The benchmark's workload (4096^2, 8 sinkers, eta 1e6/1, T = 64, h = k = 8):
    one outer iteration compared with the oracle over the whole field."""
    p = I.smoother_workload(4096, 2)
    shifts = I.random_shifts(1, 64, 64, 3)
    kw = dict(tile_x=64, tile_y=64, k=k, halo=k, shifts=shifts)
    gx, gy = gpu_smooth(ctx, p, torch.float64, "ras", k, **kw)
    ox, oy = S.smooth(p, *p.zeros_v(), p.fx, p.fy, None, k, "ras", **kw)
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64


@pytest.mark.parametrize("k", [2, 4, 8])
def test_full_size_4096_ras_fp32_one_outer_iteration_vs_oracle(ctx, k):
    """The FP32 leg of the benchmark's workload (4096^2, 8 sinkers, eta 1e6/1,
    T = 64, h = k): one outer iteration of k FP32 sweeps from an FP64 state
    two Jacobi sweeps in, rounded to FP32 (the oracle takes the same rounded
    inputs), against the FP64 oracle over the whole field, k * 1e-5."""
    p = I.smoother_workload(4096, 2)
    bx, by = S.rhs(p, p.fx, p.fy)
    vx, vy = p.zeros_v()
    for _ in range(2):
        vx, vy = S.jacobi(p, bx, by, 0.7, vx, vy)
    p32 = I.Problem(p.nx, p.ny, p.dx, p.dy, as_dtype(p.eta_c, torch.float32), as_dtype(p.eta_n, torch.float32),
                    as_dtype(p.fx, torch.float32), as_dtype(p.fy, torch.float32))
    vx, vy = as_dtype(vx, torch.float32), as_dtype(vy, torch.float32)
    shifts = I.random_shifts(1, 64, 64, 3)
    kw = dict(tile_x=64, tile_y=64, k=k, halo=k, shifts=shifts)
    gx, gy = gpu_smooth(ctx, p32, torch.float32, "ras", k, vx, vy, **kw)
    ox, oy = S.smooth(p32, vx, vy, p32.fx, p32.fy, None, k, "ras", **kw)
    assert normwise(gx, ox) <= k * TOL32 and normwise(gy, oy) <= k * TOL32


@pytest.mark.parametrize("kt,h", [(4, 4), (3, 1), (0, 2)])
def test_ras_outer_entry_point_out_of_place(ctx, kt, h):
    from paper_2509_19061_amd import api, fields
    p = ragged_problem(150, 110, 28, 1e5)
    vx0, vy0 = I.random_velocity(p, 29, 1e-3)
    dp = fields.DeviceProblem(p, torch.float64)
    vx, vy = dp.velocity(vx0, vy0)
    ox, oy = dp.field(np.full((p.ny + 1, p.nx + 1), 7.0)), dp.field(np.full((p.ny + 1, p.nx + 1), 7.0))
    api.ras_outer(ctx, torch.float64, dp.grid, vx, vy, dp.eta_c, dp.eta_n, dp.fx, dp.fy, ox, oy, 0.7, 48, 40, h, kt,
                  17, 33)
    torch.cuda.synchronize()
    bx, by = S.rhs(p, p.fx, p.fy)
    rx, ry = S.ras_outer(p, bx, by, 0.7, 48, 40, h, kt, 17, 33, vx0, vy0)
    assert normwise(dp.get_vx(ox), rx) <= TOL64 and normwise(dp.get_vy(oy), ry) <= TOL64
    # inputs untouched, walls of the output written
    assert np.array_equal(dp.get_vx(vx), vx0) and np.array_equal(dp.get_vy(vy), vy0)
    assert np.all(dp.get_vx(ox)[:, [0, -1]] == 0) and np.all(dp.get_vy(oy)[[0, -1], :] == 0)


def test_ras_streaming_tall_tiles_and_many_tiles_per_workgroup(ras_ctx):
    """Tiles stacked in one workgroup (streamed without draining), small tiles
    so that workgroups hold several, rectangular tiles, thin halo."""
    p = ragged_problem(301, 257, 30, 1e6)
    vx0, vy0 = I.random_velocity(p, 31, 1e-3)
    for (tx, ty, k, h) in [(16, 8, 3, 1), (40, 24, 4, 0), (64, 64, 6, 2), (13, 29, 2, 2)]:
        shifts = I.random_shifts(4, tx, ty, tx + ty)
        kw = dict(tile_x=tx, tile_y=ty, k=k, halo=h, shifts=shifts)
        gx, gy = gpu_smooth(ras_ctx, p, torch.float64, "ras", 2 * k + 1, vx0, vy0, **kw)
        ox, oy = S.smooth(p, vx0, vy0, p.fx, p.fy, None, 2 * k + 1, "ras", **kw)
        assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64, (tx, ty, k, h)


def test_ras_large_k_falls_back_to_window_kernel(ctx):
    p = ragged_problem(150, 140, 32, 1e3)
    vx0, vy0 = I.random_velocity(p, 33, 1e-3)
    shifts = I.random_shifts(2, 64, 64, 34)
    kw = dict(tile_x=64, tile_y=64, k=16, halo=2, shifts=shifts)
    gx, gy = gpu_smooth(ctx, p, torch.float64, "ras", 20, vx0, vy0, **kw)
    ox, oy = S.smooth(p, vx0, vy0, p.fx, p.fy, None, 20, "ras", **kw)
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64


def test_8192_ras_equals_fused_jacobi_bitwise(ctx):
    """Largest workload size (8192^2, the refinement workload): with h >= k - 1
    an outer iteration is k Jacobi sweeps exactly, at any size, so the streaming
    kernel must reproduce the fused kernel (oracle-checked at smaller sizes)
    bit for bit; two outer iterations with different shifts."""
    from paper_2509_19061_amd import api, fields
    p = I.lognormal_background_workload(8192, 4, 16)
    dp = fields.DeviceProblem(p, torch.float64)
    shifts = I.random_shifts(2, 64, 64, 9)
    vx, vy = dp.velocity(*I.random_velocity(p, 3, 1e-3))
    wx, wy = vx.clone(), vy.clone()
    api.smooth(ctx, torch.float64, dp.grid, vx, vy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, 8, "ras",
               tile_x=64, tile_y=64, k=4, halo=4, shifts=shifts)
    api.smooth(ctx, torch.float64, dp.grid, wx, wy, None, dp.eta_c, dp.eta_n, dp.fx, dp.fy, 8, "jacobi_fused")
    torch.cuda.synchronize()
    assert torch.equal(vx, wx) and torch.equal(vy, wy)


@pytest.mark.parametrize("k", [2, 4, 8])
def test_thin_overlap_ras_benchmark_configurations(ctx, k):
    """The halo-0 RAS configurations the benchmark times (64 x 64 tiles,
    k = 2, 4, 8, shift stream seed 3), with the kernel choice the benchmark
    gets, against the oracle on a grid of several tiles with a ragged edge."""
    p = ragged_problem(200, 136, 50 + k, 1e6)
    vx0, vy0 = I.random_velocity(p, 60 + k, 1e-2)
    sweeps = 3 * k
    shifts = I.random_shifts(3, 64, 64, 3)
    gx, gy = gpu_smooth(ctx, p, torch.float64, "ras", sweeps, vx0, vy0, tile_x=64, tile_y=64, k=k, halo=0,
                        shifts=shifts)
    ox, oy = S.smooth(p, vx0, vy0, p.fx, p.fy, None, sweeps, "ras", tile_x=64, tile_y=64, k=k, halo=0,
                      shifts=shifts)
    assert normwise(gx, ox) <= TOL64 and normwise(gy, oy) <= TOL64
