"""Host-side tests of the continuous-batching scheduler with a mock executor:
admission by budget, queueing, FIFO order, slot reuse, step counts."""

import pytest

from paper_2406_17981_amd.serve import Executor, Request, Server, latency_summary, poisson_requests


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class MockExecutor(Executor):
    """Memory = 10 units per grid point count class; every step costs 1 ms of
    fake time; records the server's view of reserved memory."""

    def __init__(self, clock, server_ref, sizes):
        self.clock = clock
        self.server_ref = server_ref
        self.sizes = sizes
        self.log = []
        self.steps = {}

    def bytes_needed(self, req):
        return self.sizes[req.n], 5

    def admit(self, req):
        srv = self.server_ref[0]
        assert srv.reserved <= srv.budget
        self.log.append(("admit", req.rid, self.clock()))
        self.steps[req.rid] = 0
        return req

    def step(self, slots):
        srv = self.server_ref[0]
        assert srv.reserved <= srv.budget
        for r in slots:
            self.steps[r.rid] += 1
        self.clock.t += 1e-3

    def finish(self, slot):
        self.log.append(("finish", slot.rid, self.clock()))
        return dict(steps=self.steps[slot.rid])

    def release(self, slot):
        pass


def _make(budget, sizes, max_active=256):
    clock = FakeClock()
    ref = [None]
    ex = MockExecutor(clock, ref, sizes)
    srv = Server(ex, budget, max_active=max_active, clock=clock, sleep=clock.sleep)
    ref[0] = srv
    return srv, ex, clock


def test_all_requests_finish_with_their_step_counts():
    reqs = poisson_requests(401, 200.0, 60, steps=7)
    sizes = {r.n: 10 for r in reqs}
    srv, ex, _ = _make(10_000, sizes)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(60))
    for r in done:
        assert r.result["steps"] == 7
        assert r.done >= r.admitted >= r.arrival
    s = latency_summary(done)
    assert s["requests"] == 60 and s["p99_s"] >= s["p50_s"] > 0


def test_budget_limits_concurrency_and_queues_fifo():
    reqs = [Request(rid=i, arrival=0.0001 * i, n=(8, 8), k=1.0, steps=5) for i in range(10)]
    srv, ex, _ = _make(budget=3 * 10 + 5, sizes={(8, 8): 10})
    done = srv.run(reqs)
    assert max(srv.batch_sizes) == 3          # only three fit at once
    assert srv.peak_reserved <= srv.budget
    admits = [rid for ev, rid, _ in ex.log if ev == "admit"]
    assert admits == list(range(10))          # first come, first served
    assert len(done) == 10


def test_continuous_batching_admits_between_steps():
    # a long request is running when short ones arrive: they join it mid-chain
    reqs = [Request(rid=0, arrival=0.0, n=(4, 4), k=1.0, steps=50),
            Request(rid=1, arrival=0.010, n=(4, 4), k=1.0, steps=5),
            Request(rid=2, arrival=0.020, n=(4, 4), k=1.0, steps=5)]
    srv, ex, _ = _make(budget=1000, sizes={(4, 4): 10})
    done = {r.rid: r for r in srv.run(reqs)}
    assert done[1].admitted < done[0].done and done[1].done < done[0].done
    assert 2 in srv.batch_sizes and 1 in srv.batch_sizes


def test_max_active_slots_are_reused():
    reqs = [Request(rid=i, arrival=0.0, n=(4, 4), k=1.0, steps=3) for i in range(7)]
    srv, ex, _ = _make(budget=10**9, sizes={(4, 4): 10}, max_active=2)
    done = srv.run(reqs)
    assert len(done) == 7 and max(srv.batch_sizes) == 2


def test_request_larger_than_budget_fails_alone():
    """An oversized request ends with an error result; the requests around it
    are served normally and every byte is returned."""
    reqs = [Request(rid=0, arrival=0.0, n=(8, 8), k=1.0, steps=3),
            Request(rid=1, arrival=0.0, n=(64, 64), k=1.0, steps=3),
            Request(rid=2, arrival=0.001, n=(8, 8), k=1.0, steps=3)]
    srv, ex, _ = _make(budget=100, sizes={(64, 64): 1000, (8, 8): 10})
    done = {r.rid: r for r in srv.run(reqs)}
    assert done[1].status == "error" and "budget" in done[1].result["error"]
    assert done[0].status == "ok" and done[2].status == "ok"
    assert done[0].result["steps"] == 3 and done[2].result["steps"] == 3
    assert srv.reserved == 0 and srv.failed == 1


class FailingExecutor(MockExecutor):
    """Admission of `bad_admit` raises (an allocation failure); the step of
    `bad_step` fails at its second step."""

    def __init__(self, *a, bad_admit=(), bad_step=(), **k):
        super().__init__(*a, **k)
        self.bad_admit, self.bad_step = set(bad_admit), set(bad_step)
        self.released = []

    def admit(self, req):
        if req.rid in self.bad_admit:
            raise MemoryError("hipMalloc: out of memory (injected)")
        return super().admit(req)

    def step(self, slots):
        super().step(slots)
        return [(i, "HIP_ERROR (injected)") for i, r in enumerate(slots)
                if r.rid in self.bad_step and self.steps[r.rid] == 2]

    def release(self, slot):
        self.released.append(slot.rid)


def _make_failing(budget, sizes, **kw):
    clock = FakeClock()
    ref = [None]
    ex = FailingExecutor(clock, ref, sizes, **kw)
    srv = Server(ex, budget, clock=clock, sleep=clock.sleep)
    ref[0] = srv
    return srv, ex, clock


def test_admission_and_step_failures_are_isolated():
    """One admission raising and one request's step failing end those two
    requests with error results (the failed step's slot is released and its
    memory returned); the rest finish with their full step counts."""
    reqs = [Request(rid=i, arrival=0.001 * i, n=(8, 8), k=1.0, steps=4) for i in range(6)]
    srv, ex, _ = _make_failing(budget=1000, sizes={(8, 8): 10}, bad_admit={1}, bad_step={3})
    done = {r.rid: r for r in srv.run(reqs)}
    assert len(done) == 6
    assert done[1].status == "error" and "out of memory" in done[1].result["error"]
    assert done[3].status == "error" and done[3].result["steps_done"] == 1 and "injected" in done[3].result["error"]
    for rid in (0, 2, 4, 5):
        assert done[rid].status == "ok" and done[rid].result["steps"] == 4
    assert 3 in ex.released and 1 not in ex.released
    assert srv.reserved == 0 and srv.failed == 2
    summ = latency_summary(list(done.values()))
    assert summ["requests"] == 4 and summ["failed"] == 2


def test_cancellation_and_deadlines():
    """A cancelled queued request never runs; a cancelled active one stops at
    the next step boundary and is released; a request past its deadline is
    cancelled; the others are unaffected."""
    reqs = [Request(rid=0, arrival=0.0, n=(8, 8), k=1.0, steps=50),
            Request(rid=1, arrival=0.0, n=(8, 8), k=1.0, steps=5),
            Request(rid=2, arrival=0.0, n=(8, 8), k=1.0, steps=50),
            Request(rid=3, arrival=0.0, n=(8, 8), k=1.0, steps=500, deadline=0.1),
            Request(rid=4, arrival=0.0, n=(8, 8), k=1.0, steps=5)]
    srv, ex, clock = _make_failing(budget=60, sizes={(8, 8): 10})
    orig_step = ex.step

    def step(slots):
        if ex.steps.get(0) == 10:
            srv.cancel(0)   # active
            srv.cancel(2)   # ... and another one
        return orig_step(slots)
    ex.step = step
    srv.cancel(1)           # cancelled before it is admitted
    done = {r.rid: r for r in srv.run(reqs)}
    assert done[1].status == "cancelled" and 1 not in ex.steps
    assert done[0].status == "cancelled" and done[0].result["steps_done"] == 11
    assert done[2].status == "cancelled" and done[2].result["steps_done"] == 11
    assert done[3].status == "cancelled" and done[3].result["steps_done"] < 500
    assert done[4].status == "ok" and done[4].result["steps"] == 5
    assert srv.reserved == 0 and srv.cancelled == 4


def test_poisson_stream_statistics():
    reqs = poisson_requests(401, 200.0, 4000)
    gaps = [b.arrival - a.arrival for a, b in zip(reqs, reqs[1:])]
    assert abs(sum(gaps) / len(gaps) - 1 / 200.0) < 0.1 / 200.0
    d2 = sum(1 for r in reqs if len(r.n) == 2)
    assert 0.45 < d2 / len(reqs) < 0.55
    assert all(0.5 <= r.k <= 1.5 for r in reqs)


class PoolingExecutor(MockExecutor):
    """Keeps released requests' memory as an idle pool per grid (as the GPU
    executor keeps plans) and checks that admissions never exceed the budget
    with the pool counted."""

    def __init__(self, clock, server_ref, sizes, pool_bytes):
        super().__init__(clock, server_ref, sizes)
        self.pool_bytes = pool_bytes
        self.idle = {}          # grid -> count of idle entries
        self.trims = 0
        self.reuses = 0

    def idle_bytes(self, req=None):
        total = sum(self.idle.values()) * self.pool_bytes
        if req is not None and self.idle.get(req.n):
            total -= self.pool_bytes
        return total

    def trim(self, req=None):
        self.trims += 1
        keep = req.n if req is not None else None
        self.idle = {k: (1 if k == keep and v else 0) for k, v in self.idle.items()}

    def admit(self, req):
        srv = self.server_ref[0]
        assert srv.reserved + self.idle_bytes(req) <= srv.budget
        if self.idle.get(req.n):
            self.idle[req.n] -= 1
            self.reuses += 1
        return super().admit(req)

    def release(self, slot):
        self.idle[slot.n] = self.idle.get(slot.n, 0) + 1


@pytest.mark.parametrize("grids,reuse,trim", [([(4, 4, 4)], True, False),
                                              ([(4, 4, 4), (8, 8), (2, 2, 2, 2)], False, True)])
def test_idle_pool_counts_against_the_budget_and_is_trimmed(grids, reuse, trim):
    # each request holds 10 units while active (plus 5 during admission); a
    # released one leaves 4 idle units behind for its grid; the budget fits two
    # active requests and an admission, but not two idle entries of other grids
    # besides: on one grid every later admission takes over an idle entry, with
    # three grids in turn admissions must trim the others' entries
    reqs = [Request(rid=i, arrival=0.0001 * i, n=grids[i % len(grids)], k=1.0, steps=3) for i in range(12)]
    clock = FakeClock()
    ref = [None]
    ex = PoolingExecutor(clock, ref, {g: 10 for g in grids}, pool_bytes=4)
    srv = Server(ex, 2 * 10 + 5 + 3, clock=clock, sleep=clock.sleep)
    ref[0] = srv
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(12))
    assert (ex.reuses > 0) == reuse
    assert (ex.trims > 0) == trim
    assert srv.peak_reserved <= srv.budget


class DelayedExecutor(MockExecutor):
    """Results become ready only after two more calls of finish_ready (as an
    asynchronous copy that lands later); finish must not be called before."""

    def __init__(self, clock, server_ref, sizes):
        super().__init__(clock, server_ref, sizes)
        self.pending = {}

    def finish_start(self, slot):
        self.pending[slot.rid] = 2

    def finish_ready(self, slot):
        self.pending[slot.rid] -= 1
        return self.pending[slot.rid] <= 0

    def finish_wait(self, slot):
        self.pending[slot.rid] = 0

    def finish(self, slot):
        assert self.pending.pop(slot.rid) <= 0
        return super().finish(slot)


def test_asynchronous_completion_keeps_slots_and_memory_until_ready():
    reqs = [Request(rid=i, arrival=0.0, n=(4, 4), k=1.0, steps=2 + i) for i in range(5)]
    clock = FakeClock()
    ref = [None]
    ex = DelayedExecutor(clock, ref, {(4, 4): 10})
    srv = Server(ex, 2 * 10 + 5, max_active=2, clock=clock, sleep=clock.sleep)
    ref[0] = srv
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(5))
    assert not ex.pending
    assert max(srv.batch_sizes) <= 2 and srv.peak_reserved <= srv.budget
    for r in done:
        assert r.result["steps"] == r.steps
