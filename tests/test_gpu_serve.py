"""Continuous batching on the GPU: solves that join a running batch, and a
served Poisson mix, give the same result bit for bit as each solve alone."""
import numpy as np
import pytest
import torch

from paper_2509_19061_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2509_19061_amd import api
    c = api.Context(0)
    yield c
    c.close()


def problems():
    rng = np.random.default_rng(50)
    return [I.instance_problem(n, rng) for n in (64, 128, 96, 64)]


def alone(ctx, p, mode, tol=1e-8, **opts):
    from paper_2509_19061_amd import api, fields
    dp = fields.DeviceProblem(p, torch.float64)
    m = api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n, **opts)
    vx, vy = dp.velocity()
    rep = m.solve(mode, vx, vy, None, dp.fx, dp.fy, tol=tol, max_iters=2000)
    out = (dp.get_vx(vx), dp.get_vy(vy), rep)
    m.close()
    return out


@pytest.mark.parametrize("coarsest", [8, 32])
@pytest.mark.parametrize("mode", ["f64", "f32_refined"])
def test_solves_joining_midway_match_alone(ctx, mode, coarsest):
    """With coarsest 32 the batch mixes coarsest levels of 1984 (64^2, 128^2)
    and 1104 (96^2 -> 24^2) unknowns in one coarse-solve launch."""
    from paper_2509_19061_amd import api, fields
    probs = problems()
    ref = [alone(ctx, p, mode, coarsest=coarsest) for p in probs]
    b = api.Batch(ctx, mode, 3)
    dps = [fields.DeviceProblem(p, torch.float64) for p in probs]
    mgs = [api.MG(ctx, d.grid, d.eta_c, d.eta_n, coarsest=coarsest) for d in dps]
    vs = [d.velocity() for d in dps]
    results, slot_of = {}, {}

    def add(q):
        slot_of[b.add(mgs[q], vs[q][0], vs[q][1], None, dps[q].fx, dps[q].fy, tol=1e-8, max_iters=2000)] = q

    add(0)
    add(1)
    steps, nxt, joined = 0, 2, 0
    while len(results) < len(probs):
        for slot, rep in b.step(3):
            results[slot_of.pop(slot)] = rep
        steps += 1
        if steps >= 2 and nxt < len(probs) and b.count() < 3:  # join while others iterate
            joined += b.count() > 0
            add(nxt)
            nxt += 1
    b.close()
    assert joined >= 1
    for q in range(len(probs)):
        rx, ry, rrep = ref[q]
        assert results[q]["converged"] and results[q]["iterations"] == rrep["iterations"]
        assert np.array_equal(dps[q].get_vx(vs[q][0]), rx) and np.array_equal(dps[q].get_vy(vs[q][1]), ry)
        assert results[q]["ev"] == rrep["ev"]
    for m in mgs:
        m.close()


@pytest.mark.parametrize("mode", ["f64", "f32_refined"])
def test_served_poisson_mix_matches_alone(ctx, mode):
    from paper_2509_19061_amd import serve
    reqs = serve.poisson_requests(10, 40.0, [64, 128, 256], seed=7)
    for r in reqs:
        r.payload = I.instance_problem(r.n, np.random.default_rng(r.seed))
    be = serve.GpuBackend(ctx, mode, 6, tol=1e-8, max_iters=2000, keep_results=True)
    res = serve.Server(be, 8 << 30, max_slots=6, iters_per_step=2).run(reqs)
    be.close()
    s = res.summary()
    assert s["completed"] == 10 and s["all_converged"]
    assert s["admitted_while_busy"] >= 1 and s["max_inflight"] >= 2
    for r in reqs:
        rx, ry, _ = alone(ctx, r.payload, mode)
        gx, gy = be.results[r.rid]
        assert np.array_equal(gx, rx) and np.array_equal(gy, ry), r.rid


def test_batch_errors(ctx):
    from paper_2509_19061_amd import api, fields
    p = problems()[0]
    dp = fields.DeviceProblem(p, torch.float64)
    m = api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n)
    m2 = api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n, omega=0.6)
    m3 = api.MG(ctx, dp.grid, dp.eta_c, dp.eta_n)
    b = api.Batch(ctx, "f64", 1)
    vx, vy = dp.velocity()
    b.add(m, vx, vy, None, dp.fx, dp.fy)
    with pytest.raises(api.StkError) as e:  # no free slot
        b.add(m3, *dp.velocity(), None, dp.fx, dp.fy)
    assert e.value.code == api.EINVAL
    with pytest.raises(api.StkError) as e:  # handle busy
        m.close()
    assert e.value.code == api.EINVAL
    b2 = api.Batch(ctx, "f64", 2)
    with pytest.raises(api.StkError):  # already in a batch
        b2.add(m, *dp.velocity(), None, dp.fx, dp.fy)
    b2.add(m3, *dp.velocity(), None, dp.fx, dp.fy)
    with pytest.raises(api.StkError):  # smoothing options differ from the batch's
        b2.add(m2, *dp.velocity(), None, dp.fx, dp.fy)
    b.close()
    b2.close()
    for h in (m, m2, m3):
        h.close()


@pytest.mark.parametrize("mode", ["f64", "f32_refined"])
def test_hierarchy_built_on_a_setup_stream_and_bound_solves_the_same(ctx, mode):
    """A hierarchy built on another context (its own stream, as the serving
    loop's setup thread does) and moved with stk_mg_bind gives the bits of one
    built on the solving context; a handle in a batch cannot be moved."""
    from paper_2509_19061_amd import api, fields
    p = problems()[1]
    rx, ry, rrep = alone(ctx, p, mode)
    s2 = torch.cuda.Stream()
    ctx2 = api.Context(0, stream=s2)
    with torch.cuda.stream(s2):
        dp = fields.DeviceProblem(p, torch.float64)
        vx, vy = dp.velocity()
    m = api.MG(ctx2, dp.grid, dp.eta_c, dp.eta_n)
    m.bind(ctx, mode)
    torch.cuda.synchronize()
    b = api.Batch(ctx, mode, 1)
    b.add(m, vx, vy, None, dp.fx, dp.fy, tol=1e-8, max_iters=2000)
    with pytest.raises(api.StkError) as e:
        m.bind(ctx2, mode)
    assert e.value.code == api.EINVAL
    done = []
    while not done:
        done = b.step(4)
    b.close()
    assert done[0][1]["iterations"] == rrep["iterations"]
    assert np.array_equal(dp.get_vx(vx), rx) and np.array_equal(dp.get_vy(vy), ry)
    m.close()
    ctx2.close()
