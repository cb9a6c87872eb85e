"""GPU inexact Uzawa iteration (lithostatic start, pressure update, cycles) vs
the CPU oracle (oracle/uzawa.py), through the C ABI.

Tolerances: the lithostatic and pressure-update passes are a few roundings
per cell (1e-13 normwise).  The Uzawa cycles run the V-cycle, whose GPU and
oracle hierarchies agree to ~1e-11 per cycle (the coarsest solves differ in
rounding, amplified by the coarse condition number), hence 1e-9 after a few
cycles.
"""
import numpy as np
import pytest
import torch

from gpu_util import normwise
from oracle import mg as OM
from oracle import stokes as S
from oracle import uzawa as U
from paper_2509_19061_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2509_19061_amd import api
    c = api.Context(0)
    yield c
    c.close()


def sinkers(nx, ny, seed, contrast):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.2, 0.8, size=(3, 2))
    r = rng.uniform(0.06, 0.12, size=3)
    return I.sinker_problem(nx, ny, [(float(c[k, 0]), float(c[k, 1]), float(r[k])) for k in range(3)], contrast, 1.0)


def dev(p, align=64):
    from paper_2509_19061_amd import fields
    return fields.DeviceProblem(p, torch.float64, align=align)


@pytest.mark.parametrize("nx,ny", [(2, 2), (64, 64), (130, 70), (257, 300)])
def test_litho_matches_oracle(ctx, nx, ny):
    from paper_2509_19061_amd import api
    p = sinkers(nx, ny, nx * 7 + ny, 1e3)
    rng = np.random.default_rng(nx + ny)
    p.fy = p.fy * rng.uniform(0.5, 1.5, size=p.fy.shape)   # varies along x too
    d = dev(p)
    pt = d.field()
    api.litho_pressure(ctx, d.grid, d.fy, pt)
    torch.cuda.synchronize()
    got = d.get_cell(pt)
    assert normwise(got, U.litho(p, p.fy)) <= 1e-13
    assert abs(got.mean()) <= 1e-13 * np.abs(got).max()
    # the pressure row past the cells (the array's last row) is untouched
    assert float(pt[ny].abs().max()) == 0.0


@pytest.mark.parametrize("nx,ny,omega_p", [(2, 2, 0.6), (64, 64, 0.6), (130, 97, 1.3), (300, 260, 0.6)])
def test_pressure_update_matches_oracle(ctx, nx, ny, omega_p):
    from paper_2509_19061_amd import api
    p = sinkers(nx, ny, nx + 3 * ny, 1e4)
    vx, vy = I.random_velocity(p, 11, 1e-2)
    p0 = I.random_pressure(p, 12)
    d = dev(p)
    tx, ty = d.velocity(vx, vy)
    pt = d.field(p0)
    api.uzawa_pressure(ctx, d.grid, tx, ty, d.eta_c, omega_p, pt)
    torch.cuda.synchronize()
    ref = U.pressure_update(p, vx, vy, p0, omega_p)
    got = d.get_cell(pt)
    assert normwise(got, ref) <= 1e-13
    assert abs(got.mean()) <= 1e-13 * np.abs(got).max()
    # the call is deterministic bit for bit
    pt2 = d.field(p0)
    api.uzawa_pressure(ctx, d.grid, tx, ty, d.eta_c, omega_p, pt2)
    torch.cuda.synchronize()
    assert torch.equal(pt, pt2)


# align 128 at nx = 128: a padded row stride (256 instead of 192)
@pytest.mark.parametrize("nx,ny,contrast,vcycles,align", [(64, 64, 1e2, 1, 64), (96, 64, 1e3, 2, 64),
                                                         (128, 128, 1e4, 1, 64), (128, 128, 1e4, 1, 128)])
def test_uzawa_cycles_match_oracle(ctx, nx, ny, contrast, vcycles, align):
    from paper_2509_19061_amd import api
    p = sinkers(nx, ny, nx + ny + 1, contrast)
    d = dev(p, align)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    p0 = U.litho(p, p.fy)
    vx, vy = d.velocity()
    pt = d.field(p0)
    cycles = 8
    rep, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True,
                                omega_p=0.6, vcycles=vcycles, tol=0.0, max_cycles=cycles)
    assert rep["cycles"] == cycles and not rep["converged"]
    levels = OM.hierarchy(p, coarsest=8)
    ox, oy, op, oh = U.uzawa(levels, p, p.fx, p.fy, *p.zeros_v(), p0, omega_p=0.6, vcycles=vcycles, tol=0.0,
                             max_cycles=cycles)
    assert normwise(d.get_vx(vx), ox) <= 1e-9 and normwise(d.get_vy(vy), oy) <= 1e-9
    assert normwise(d.get_cell(pt), op) <= 1e-9
    np.testing.assert_allclose(hist, oh, rtol=1e-8)
    assert rep["e"] == hist[-1]
    m.close()


def test_uzawa_strides_agree_bitwise(ctx):
    """The result does not depend on the row stride (padding): 192 and 256
    give the same bits."""
    from paper_2509_19061_amd import api
    p = sinkers(128, 96, 17, 1e3)
    res = []
    for align in (64, 128):
        d = dev(p, align)
        assert d.ld == (192 if align == 64 else 256)
        m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
        vx, vy = d.velocity()
        pt = d.field()
        api.litho_pressure(ctx, d.grid, d.fy, pt)
        _, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True, tol=0.0,
                                  max_cycles=6)
        res.append((d.get_vx(vx), d.get_vy(vy), d.get_cell(pt), hist))
        m.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_uzawa_constant_viscosity_two_cycles_exact(ctx):
    """Exact velocity solves (one level: the dense coarsest solve) and
    constant viscosity: the Schur complement is I/(2 eta) on mean-zero
    pressures, so omega_p = 2 reaches the saddle-point solution in two cycles."""
    from paper_2509_19061_amd import api
    nx = ny = 32
    p = I.sinker_problem(nx, ny, [], 7.0, 7.0)
    rng = np.random.default_rng(5)
    p.fx = rng.standard_normal(p.fx.shape)
    p.fy = rng.standard_normal(p.fy.shape)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n, coarsest=64)
    assert m.info()["levels"] == 1
    vx, vy = d.velocity()
    pt = d.field()
    rep, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, omega_p=2.0, tol=1e-11,
                                max_cycles=10)
    assert rep["converged"] and rep["cycles"] == 2, hist
    assert hist[1] > 1e-3
    m.close()


def test_uzawa_converges_from_litho(ctx):
    from paper_2509_19061_amd import api
    p = sinkers(64, 64, 9, 1e2)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    vx, vy = d.velocity()
    pt = d.field()
    api.litho_pressure(ctx, d.grid, d.fy, pt)
    rep, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, omega_p=0.6, tol=1e-8,
                                max_cycles=2000)
    assert rep["converged"] and hist[-1] <= 1e-8 < hist[0]
    # the result solves both blocks: recompute E in the oracle
    e = S.energy(p, d.get_vx(vx), d.get_vy(vy), p.fx, p.fy, d.get_cell(pt))
    assert e[3] <= 1.01e-8
    m.close()


def test_uzawa_argument_errors(ctx):
    from paper_2509_19061_amd import api
    from paper_2509_19061_amd._lib import Grid
    p = sinkers(64, 64, 1, 1e2)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    vx, vy = d.velocity()
    pt = d.field()
    before = pt.clone()
    with pytest.raises(api.StkError) as e:
        api.uzawa_pressure(ctx, d.grid, vx, vy, d.eta_c, 0.0, pt)
    assert e.value.code == api.EINVAL
    other = Grid(32, 64, d.ld, 1 / 32, 1 / 64)
    with pytest.raises(api.StkError) as e:
        api.uzawa_solve(m, other, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy)
    assert e.value.code == api.EINVAL
    with pytest.raises(api.StkError) as e:
        api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, vcycles=0)
    assert e.value.code == api.EINVAL
    torch.cuda.synchronize()
    assert torch.equal(pt, before)
    # not converged: arrays and report still written
    rep, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True,
                                max_cycles=2)
    assert rep["cycles"] == 2 and not rep["converged"] and len(hist) == 3
    m.close()


@pytest.mark.parametrize("nx,contrast,align", [(64, 1e4, 64), (128, 1e3, 128)])
def test_continuation_matches_oracle(ctx, nx, contrast, align):
    """Four continuation stages of three cycles each, then four cycles of the
    true system; the second case has a padded stride (256 at nx = 128)."""
    from paper_2509_19061_amd import api
    p = sinkers(nx, nx, nx + 5, contrast)
    d = dev(p, align)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    p0 = U.litho(p, p.fy)
    vx, vy = d.velocity()
    pt = d.field(p0)
    rep, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True, tol=0.0,
                                max_cycles=16, stages=4, stage_cycles=3)
    assert rep["cycles"] == 16
    ox, oy, op, oh = U.uzawa_continuation(p, p.fx, p.fy, *p.zeros_v(), p0, stages=4, stage_cycles=3, tol=0.0,
                                          max_cycles=16)
    assert normwise(d.get_vx(vx), ox) <= 1e-9 and normwise(d.get_vy(vy), oy) <= 1e-9
    assert normwise(d.get_cell(pt), op) <= 1e-9
    np.testing.assert_allclose(hist, oh, rtol=1e-8)
    m.close()


def test_continuation_exact_solves_match_oracle(ctx):
    """One-level hierarchies (exact velocity solves): stage 0 runs on the
    constant viscosity min(eta_c), where omega_p = 2 reaches that system's
    saddle point in two cycles; the oracle's pin of this case is the
    assembled saddle-point solve."""
    from paper_2509_19061_amd import api
    p = sinkers(32, 32, 3, 1e3)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n, coarsest=64)
    vx, vy = d.velocity()
    pt = d.field()
    rep, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True, tol=0.0,
                                omega_p=2.0, max_cycles=6, stages=2, stage_cycles=2)
    ox, oy, op, oh = U.uzawa_continuation(p, p.fx, p.fy, *p.zeros_v(), np.zeros((32, 32)), stages=2,
                                          stage_cycles=2, omega_p=2.0, tol=0.0, max_cycles=6, coarsest=64)
    assert normwise(d.get_vx(vx), ox) <= 1e-9 and normwise(d.get_vy(vy), oy) <= 1e-9
    assert normwise(d.get_cell(pt), op) <= 1e-9
    np.testing.assert_allclose(hist, oh, rtol=1e-8)
    m.close()


def test_continuation_options_rejected(ctx):
    from paper_2509_19061_amd import api
    p = sinkers(64, 64, 1, 1e2)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    vx, vy = d.velocity()
    pt = d.field()
    for bad in (dict(stages=-1), dict(stages=2, stage_cycles=-3)):
        with pytest.raises(api.StkError) as e:
            api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, **bad)
        assert e.value.code == api.EINVAL
    m.close()


def test_anderson_depth_zero_equals_plain_cycles_bitwise(ctx):
    from paper_2509_19061_amd import api
    p = sinkers(96, 64, 21, 1e3)
    res = []
    for depth in (None, 0):
        d = dev(p)
        m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
        vx, vy = d.velocity()
        pt = d.field()
        api.litho_pressure(ctx, d.grid, d.fy, pt)
        if depth is None:
            _, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True,
                                      tol=0.0, max_cycles=5)
        else:
            _, hist = api.uzawa_anderson(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, depth=0,
                                         allow_notconv=True, tol=0.0, max_cycles=5)
        res.append((d.get_vx(vx), d.get_vy(vy), d.get_cell(pt), hist))
        m.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


# align 128 at nx = 128: a padded row stride (256 instead of 192)
@pytest.mark.parametrize("nx,ny,contrast,depth,align", [(64, 64, 1e3, 3, 64), (96, 80, 1e2, 5, 64),
                                                       (128, 128, 1e3, 3, 128)])
def test_anderson_matches_oracle(ctx, nx, ny, contrast, depth, align):
    from paper_2509_19061_amd import api
    p = sinkers(nx, ny, nx + 2 * ny, contrast)
    d = dev(p, align)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    p0 = U.litho(p, p.fy)
    vx, vy = d.velocity()
    pt = d.field(p0)
    steps = 10
    rep, hist = api.uzawa_anderson(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, depth=depth,
                                   allow_notconv=True, tol=0.0, max_cycles=steps)
    assert rep["cycles"] == steps
    levels = OM.hierarchy(p, coarsest=8)
    ox, oy, op, oh = U.anderson(levels, p, p.fx, p.fy, *p.zeros_v(), p0, m=depth, tol=0.0, max_iters=steps)
    assert normwise(d.get_vx(vx), ox) <= 1e-8 and normwise(d.get_vy(vy), oy) <= 1e-8
    assert normwise(d.get_cell(pt), op) <= 1e-8
    np.testing.assert_allclose(hist, oh, rtol=1e-7)
    m.close()


def test_anderson_exact_third_iterate_constant_viscosity(ctx):
    """Exact velocity solves and constant viscosity: r_2 = c r_1 with
    c = 1 - omega_p/2, so the third iterate is the saddle-point solution."""
    from paper_2509_19061_amd import api
    nx = ny = 32
    p = I.sinker_problem(nx, ny, [], 3.0, 3.0)
    rng = np.random.default_rng(8)
    p.fx = rng.standard_normal(p.fx.shape)
    p.fy = rng.standard_normal(p.fy.shape)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n, coarsest=64)
    p0 = rng.standard_normal((ny, nx))
    vx, vy = d.velocity()
    pt = d.field(p0)
    rep, hist = api.uzawa_anderson(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, depth=2, omega_p=0.6,
                                   allow_notconv=True, tol=0.0, max_cycles=3)
    assert len(hist) == 4 and hist[2] > 1e-3 * hist[0]
    assert hist[3] <= 1e-10 * hist[0]
    lv = OM.hierarchy(p, coarsest=64)
    ox, oy, op, oh = U.anderson(lv, p, p.fx, p.fy, *p.zeros_v(), p0, m=2, omega_p=0.6, tol=0.0, max_iters=3)
    assert normwise(d.get_cell(pt), op) <= 1e-9 and normwise(d.get_vy(vy), oy) <= 1e-9
    m.close()


def test_anderson_options_rejected(ctx):
    from paper_2509_19061_amd import api
    p = sinkers(64, 64, 1, 1e2)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    vx, vy = d.velocity()
    pt = d.field()
    for kw, code in ((dict(depth=9), api.EINVAL), (dict(depth=-1), api.EINVAL),
                     (dict(depth=2, stages=-1), api.EINVAL), (dict(depth=2, vcycles=0), api.EINVAL)):
        with pytest.raises(api.StkError) as e:
            api.uzawa_anderson(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, **kw)
        assert e.value.code == code
    m.close()


def test_pressure_step_and_litho_full_size():
    """4096^2 (the benchmark's size): the pressure step checked on 2000 sampled
    cells, the lithostatic start by hydrostatic balance on every interior
    face."""
    from paper_2509_19061_amd import api
    c = api.Context(0)
    p = I.smoother_workload(4096)
    d = dev(p)
    rng = np.random.default_rng(31)
    vx0, vy0 = I.random_velocity(p, 32, 1e-3)
    p0 = rng.standard_normal((4096, 4096))
    vx, vy = d.velocity(vx0, vy0)
    pt = d.field(p0)
    api.uzawa_pressure(c, d.grid, vx, vy, d.eta_c, 0.6, pt)
    torch.cuda.synchronize()
    got = d.get_cell(pt)
    assert abs(got.mean()) <= 1e-12 * np.abs(got).max()
    jj, ii = rng.integers(0, 4096, 2000), rng.integers(0, 4096, 2000)
    div = (vx0[jj, ii + 1] - vx0[jj, ii]) * 4096 + (vy0[jj + 1, ii] - vy0[jj, ii]) * 4096
    step = p0[jj, ii] - 0.6 * p.eta_c[jj, ii] * div        # before the mean is removed
    shift = got[jj, ii] - step                             # = -mean, the same for every cell
    assert np.abs(shift - shift.mean()).max() <= 1e-9 * np.abs(step).max()
    full = p0 - 0.6 * p.eta_c * ((vx0[:, 1:] - vx0[:, :-1]) * 4096 + (vy0[1:] - vy0[:-1]) * 4096)
    assert abs(shift.mean() + full.mean()) <= 1e-11 * np.abs(full).max()
    # lithostatic pressure: with v = 0 the velocity residual b - M v = f - G p
    # vanishes on every interior vy face
    api.litho_pressure(c, d.grid, d.fy, pt)
    zx, zy = d.velocity()
    rx, ry = d.velocity()
    api.residual(c, torch.float64, d.grid, zx, zy, pt, d.eta_c, d.eta_n, d.fx, d.fy, rx, ry)
    torch.cuda.synchronize()
    assert float(ry[1:4096, :4096].abs().max()) <= 1e-10 * float(d.fy.abs().max())
    c.close()


@pytest.mark.parametrize("stages", [0, 2])
def test_uzawa_mixed_cycles_match_oracle(ctx, stages):
    """FP32 V-cycles on the FP64 residual: the oracle's FP64 cycles to FP32
    precision (the V-cycle is consistent: V(v, b) = v + V(0, b - M v))."""
    from paper_2509_19061_amd import api
    p = sinkers(64, 64, 41, 1e3)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    p0 = U.litho(p, p.fy)
    vx, vy = d.velocity()
    pt = d.field(p0)
    rep, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True, tol=0.0,
                                max_cycles=6, stages=stages, stage_cycles=2, mode="f32_refined")
    if stages:
        ox, oy, op, oh = U.uzawa_continuation(p, p.fx, p.fy, *p.zeros_v(), p0, stages=stages, stage_cycles=2,
                                              tol=0.0, max_cycles=6)
    else:
        ox, oy, op, oh = U.uzawa(OM.hierarchy(p), p, p.fx, p.fy, *p.zeros_v(), p0, tol=0.0, max_cycles=6)
    assert normwise(d.get_vx(vx), ox) <= 1e-5 and normwise(d.get_vy(vy), oy) <= 1e-5
    assert normwise(d.get_cell(pt), op) <= 1e-5
    np.testing.assert_allclose(hist, oh, rtol=1e-4)
    m.close()


def test_uzawa_mixed_reaches_the_fp64_solution(ctx):
    from paper_2509_19061_amd import api
    p = sinkers(128, 128, 9, 1e2)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    out = {}
    for mode in ("f64", "f32_refined"):
        vx, vy = d.velocity()
        pt = d.field()
        api.litho_pressure(ctx, d.grid, d.fy, pt)
        rep, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, tol=1e-8, max_cycles=2000,
                                    mode=mode)
        assert rep["converged"]
        out[mode] = (rep, d.get_vx(vx), d.get_vy(vy), d.get_cell(pt))
    assert out["f32_refined"][0]["cycles"] <= 1.2 * out["f64"][0]["cycles"]
    for a, b in zip(out["f32_refined"][1:], out["f64"][1:]):
        assert normwise(a, b) <= 1e-6
    m.close()


def test_uzawa_mixed_strides_agree_bitwise(ctx):
    """The FP32 V-cycle mode gives the same bits at strides 192 and 256."""
    from paper_2509_19061_amd import api
    p = sinkers(128, 128, 2, 1e2)
    res = []
    for align in (64, 128):
        d = dev(p, align)
        m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
        vx, vy = d.velocity()
        pt = d.field()
        _, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True, tol=0.0,
                                  max_cycles=4, mode="f32_refined")
        res.append((d.get_vx(vx), d.get_vy(vy), d.get_cell(pt), hist))
        if align == 64:
            m.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    m.close()


def test_anderson_mixed_matches_oracle(ctx):
    """Anderson steps over FP32 V-cycles on the FP64 residual against the
    oracle's FP64 steps: FP32 rounding of the V-cycle, passed through the
    weights (1e-4 after 6 steps)."""
    from paper_2509_19061_amd import api
    p = sinkers(64, 64, 43, 1e3)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    p0 = U.litho(p, p.fy)
    vx, vy = d.velocity()
    pt = d.field(p0)
    rep, hist = api.uzawa_anderson(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, depth=3, allow_notconv=True,
                                   tol=0.0, max_cycles=6, mode="f32_refined")
    ox, oy, op, oh = U.anderson(OM.hierarchy(p), p, p.fx, p.fy, *p.zeros_v(), p0, m=3, tol=0.0, max_iters=6)
    assert normwise(d.get_vx(vx), ox) <= 1e-4 and normwise(d.get_vy(vy), oy) <= 1e-4
    assert normwise(d.get_cell(pt), op) <= 1e-4
    np.testing.assert_allclose(hist, oh, rtol=1e-3)
    m.close()


def test_anderson_continuation_matches_oracle(ctx):
    """Two continuation stages of three Anderson steps each (history restarted
    per stage), then three steps on the true system."""
    from paper_2509_19061_amd import api
    p = sinkers(64, 64, 47, 1e4)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    p0 = U.litho(p, p.fy)
    vx, vy = d.velocity()
    pt = d.field(p0)
    rep, hist = api.uzawa_anderson(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, depth=3, allow_notconv=True,
                                   tol=0.0, max_cycles=9, stages=2, stage_cycles=3)
    assert rep["cycles"] == 9
    ox, oy, op, oh = U.anderson_continuation(p, p.fx, p.fy, *p.zeros_v(), p0, m=3, stages=2, stage_cycles=3,
                                             tol=0.0, max_iters=9)
    assert normwise(d.get_vx(vx), ox) <= 1e-8 and normwise(d.get_vy(vy), oy) <= 1e-8
    assert normwise(d.get_cell(pt), op) <= 1e-8
    np.testing.assert_allclose(hist, oh, rtol=1e-7)
    m.close()


def test_anderson_mixed_continuation_matches_oracle(ctx):
    """FP32 V-cycles, continuation stages and Anderson steps together (each
    stage hierarchy builds its own FP32 plan) against the oracle's FP64
    Anderson continuation, to the FP32 bar of the mixed tests (1e-4)."""
    from paper_2509_19061_amd import api
    p = sinkers(64, 64, 53, 1e3)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    p0 = U.litho(p, p.fy)
    vx, vy = d.velocity()
    pt = d.field(p0)
    rep, hist = api.uzawa_anderson(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, depth=3, allow_notconv=True,
                                   tol=0.0, max_cycles=8, stages=2, stage_cycles=2, mode="f32_refined")
    assert rep["cycles"] == 8
    ox, oy, op, oh = U.anderson_continuation(p, p.fx, p.fy, *p.zeros_v(), p0, m=3, stages=2, stage_cycles=2,
                                             tol=0.0, max_iters=8)
    assert normwise(d.get_vx(vx), ox) <= 1e-4 and normwise(d.get_vy(vy), oy) <= 1e-4
    assert normwise(d.get_cell(pt), op) <= 1e-4
    np.testing.assert_allclose(hist, oh, rtol=1e-3)
    m.close()


def _garbage_walls(vx, vy, nx, ny, value):
    """Write +-value on the wall velocities vx(0, .), vx(nx, .), vy(., 0), vy(., ny)."""
    vx[:ny, 0] = value
    vx[:ny, nx] = -value
    vy[0, :nx] = -value
    vy[ny, :nx] = value


def _walls_zero(vx, vy, nx, ny):
    return (float(vx[:ny, 0].abs().max()) == 0.0 and float(vx[:ny, nx].abs().max()) == 0.0
            and float(vy[0, :nx].abs().max()) == 0.0 and float(vy[ny, :nx].abs().max()) == 0.0)


def test_pressure_step_ignores_wall_values(ctx):
    """Walls are read as 0 whatever they hold: +-1e30 there gives the bits of
    the zero-wall step."""
    from paper_2509_19061_amd import api
    nx, ny = 130, 97
    p = sinkers(nx, ny, 5, 1e4)
    vx0, vy0 = I.random_velocity(p, 3, 1e-2)
    p0 = I.random_pressure(p, 4)
    d = dev(p)
    out = []
    for wall in (0.0, 1e30):
        tx, ty = d.velocity(vx0, vy0)
        _garbage_walls(tx, ty, nx, ny, wall)
        pt = d.field(p0)
        api.uzawa_pressure(ctx, d.grid, tx, ty, d.eta_c, 0.6, pt)
        torch.cuda.synchronize()
        out.append(pt.clone())
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("call", ["solve_f64", "solve_f32", "anderson_f64", "anderson_f32"])
def test_uzawa_cycles_ignore_wall_values(ctx, call):
    """The Uzawa cycles (both precision modes) and the Anderson steps give the
    same bits from a start whose walls hold +-1e30 as from zero walls, and
    write 0 on the walls."""
    from paper_2509_19061_amd import api
    nx, ny = 64, 48
    p = sinkers(nx, ny, 17, 1e3)
    d = dev(p)
    m = api.MG(ctx, d.grid, d.eta_c, d.eta_n)
    vx0, vy0 = I.random_velocity(p, 21, 1e-3)
    p0 = U.litho(p, p.fy)
    mode = "f32_refined" if call.endswith("f32") else "f64"
    res = []
    for wall in (0.0, 1e30):
        vx, vy = d.velocity(vx0, vy0)
        _garbage_walls(vx, vy, nx, ny, wall)
        pt = d.field(p0)
        if call.startswith("solve"):
            _, hist = api.uzawa_solve(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, allow_notconv=True,
                                      tol=0.0, max_cycles=4, mode=mode)
        else:
            _, hist = api.uzawa_anderson(m, d.grid, vx, vy, pt, d.eta_c, d.eta_n, d.fx, d.fy, depth=3,
                                         allow_notconv=True, tol=0.0, max_cycles=4, mode=mode)
        torch.cuda.synchronize()
        assert _walls_zero(vx, vy, nx, ny), (call, wall)
        res.append((vx.clone(), vy.clone(), pt.clone(), hist))
    for a, b in zip(res[0][:3], res[1][:3]):
        assert torch.equal(a, b), call
    assert np.array_equal(res[0][3][1:], res[1][3][1:])
    m.close()
