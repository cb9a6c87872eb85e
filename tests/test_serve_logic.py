"""Host logic of the serving loop (no GPU): admission under the HBM budget,
FIFO order, continuous batching (arrivals join while others are in flight),
rejection of requests that can never fit, latency bookkeeping."""
import numpy as np
import pytest

from paper_2509_19061_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """A request of size n needs n // 64 steps; each step advances the clock by
    dt and costs nothing else.  Records the bytes in flight at every step."""

    def __init__(self, clock, dt=0.01):
        self.clock, self.dt = clock, dt
        self.left = {}
        self.next_slot = 0
        self.used = 0
        self.trace = []
        self.order = []

    def footprint(self, r):
        return r.n * r.n

    def admit(self, r):
        slot = self.next_slot
        self.next_slot += 1
        self.left[slot] = max(1, r.n // 64)
        self.used += self.footprint(r)
        self.order.append(r.rid)
        return (slot, r), slot

    def step(self, iters):
        self.clock.t += self.dt
        self.trace.append((self.used, len(self.left)))
        out = []
        for s in list(self.left):
            self.left[s] -= 1
            if self.left[s] == 0:
                del self.left[s]
                out.append((s, {"iterations": 1, "ev": 0.0, "converged": True}))
        return out

    def release(self, handle):
        slot, r = handle
        self.used -= self.footprint(r)


def run(reqs, budget, max_slots=64):
    clk = FakeClock()
    be = FakeBackend(clk)
    res = serve.Server(be, budget, max_slots=max_slots, iters_per_step=1, clock=clk, sleep=clk.sleep).run(reqs)
    return res, be


def test_budget_is_never_exceeded_and_everything_completes():
    reqs = serve.poisson_requests(40, 50.0, [64, 128, 256], seed=1)
    budget = 3 * 256 * 256
    res, be = run(reqs, budget)
    assert len(res.done) == 40 and not res.rejected
    assert max(u for u, _ in be.trace) <= budget
    assert res.peak_bytes <= budget
    assert all(d.finished >= d.admitted >= d.arrival for d in res.done)
    assert all(d.latency == pytest.approx(d.finished - d.arrival) for d in res.done)


def test_admission_is_fifo():
    reqs = serve.poisson_requests(30, 100.0, [64, 256], seed=2)
    res, be = run(reqs, 2 * 256 * 256)
    assert be.order == sorted(be.order)  # rid order == arrival order


def test_arrivals_join_a_running_batch():
    # a long request, then short ones arriving while it runs
    reqs = [serve.Request(0, 0.0, 64 * 50, 0)] + [serve.Request(i, 0.05 * i, 64, i) for i in range(1, 6)]
    res, be = run(reqs, 10 ** 9)
    done = {d.rid: d for d in res.done}
    assert all(done[i].inflight_at_admission >= 1 for i in range(1, 6))
    assert all(done[i].finished < done[0].finished for i in range(1, 6))
    assert res.summary()["admitted_while_busy"] == 5
    assert res.max_inflight >= 2


def test_head_of_line_request_waits_for_memory():
    reqs = [serve.Request(0, 0.0, 256, 0), serve.Request(1, 0.0, 256, 1), serve.Request(2, 0.0, 64, 2)]
    res, be = run(reqs, 256 * 256 + 64 * 64)
    done = {d.rid: d for d in res.done}
    # request 1 cannot fit beside 0; request 2 (which would fit) must not overtake it
    assert done[1].admitted >= done[0].finished
    assert done[2].admitted >= done[1].admitted


def test_request_larger_than_the_budget_is_rejected():
    reqs = [serve.Request(0, 0.0, 512, 0), serve.Request(1, 0.0, 64, 1)]
    res, _ = run(reqs, 256 * 256)
    assert res.rejected == [0] and [d.rid for d in res.done] == [1]


def test_slot_limit():
    reqs = [serve.Request(i, 0.0, 128, i) for i in range(10)]
    res, be = run(reqs, 10 ** 9, max_slots=3)
    assert max(n for _, n in be.trace) <= 3 and len(res.done) == 10


def test_poisson_arrivals_have_the_requested_rate():
    reqs = serve.poisson_requests(4000, 20.0, [64], seed=3)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert gaps.mean() == pytest.approx(1 / 20.0, rel=0.05)
    assert all(r.arrival == 0.0 for r in serve.poisson_requests(5, float("inf"), [64], seed=4))


class FakeAsyncBackend(FakeBackend):
    """FakeBackend whose admission is asynchronous: a request's setup takes
    `setup` seconds of clock from prepare() and only then can it join."""

    def __init__(self, clock, dt=0.01, setup=0.05):
        super().__init__(clock, dt)
        self.setup = setup
        self.step_times = []
        self.joined = {}

    def prepare(self, r):
        return {"r": r, "ready_at": self.clock.t + self.setup}

    def ready(self, token):
        return self.clock.t >= token["ready_at"]

    def join(self, token):
        if self.clock.t < token["ready_at"]:  # the loop waits only when nothing else can run
            self.clock.t = token["ready_at"]
        self.joined[token["r"].rid] = self.clock.t
        return self.admit(token["r"])

    def step(self, iters):
        self.step_times.append(self.clock.t)
        return super().step(iters)


def test_setup_of_an_admitted_request_does_not_stall_the_batch():
    clk = FakeClock()
    be = FakeAsyncBackend(clk, dt=0.01, setup=0.05)
    reqs = [serve.Request(0, 0.0, 64 * 40, 0), serve.Request(1, 0.1, 64, 1), serve.Request(2, 0.1, 128, 2)]
    res = serve.Server(be, 10 ** 9, iters_per_step=1, clock=clk, sleep=clk.sleep).run(reqs)
    assert len(res.done) == 3
    done = {d.rid: d for d in res.done}
    # request 0 keeps stepping while 1 and 2 are being set up: steps between their arrival and their join
    during = [t for t in be.step_times if 0.1 <= t < be.joined[1]]
    assert len(during) >= 4, (be.joined, be.step_times[:20])
    assert be.joined[1] >= 0.1 + 0.05 and be.joined[2] >= be.joined[1]
    assert done[1].inflight_at_admission >= 1 and done[2].inflight_at_admission >= 1
    # the first request had nothing to overlap with: its setup was waited for
    assert be.joined[0] == pytest.approx(0.05)
