"""The serving scheduler on a modelled backend (no GPU): admission by byte
budget, continuous batching, no starvation, refusal, eviction, latency."""

import pytest

from paper_1509_07685_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-5          # every look at the clock advances it 10 us
        return self.t


class FakeEx:
    def __init__(self, key):
        self.key = key


class FakeBackend:
    """Solve time = 0.2 ms + 1 ns per mesh point per element of the batch."""

    def __init__(self, clock, max_batch=4, num_streams=2, exec_bytes=None, plan_bytes=1 << 20):
        self.clock = clock
        self.max_batch = max_batch
        self.num_streams = num_streams
        self.exec_bytes = exec_bytes or {}
        self.pbytes = plan_bytes
        self.inflight = {}
        self.launches = []
        self.created = []
        self.destroyed = []
        self.live = 0
        self.max_live_streams = 0
        self.n = 0

    def executor_bytes(self, key):
        return self.exec_bytes.get(key, 100 << 20)

    def plan_bytes(self, key):
        return self.pbytes

    def create_executor(self, key):
        self.created.append(key)
        return FakeEx(key)

    def destroy_executor(self, ex):
        self.destroyed.append(ex.key)

    def launch(self, ex, jobs, stream):
        shape = ex.key[0]
        dur = 2e-4 + 1e-9 * shape[0] * shape[1] * shape[2] * len(jobs)
        self.n += 1
        self.inflight[self.n] = self.clock.t + dur
        self.launches.append((ex.key, [j.rid for j in jobs], stream))
        self.live += 1
        self.max_live_streams = max(self.max_live_streams, self.live)
        return self.n

    def done(self, token):
        if self.clock.t >= self.inflight[token]:
            self.live -= 1
            return True
        return False

    def error(self, token):
        return None


def jobs_from(spec):
    return [serve.Job(i, t, key, 1000, 1e-15) for i, (t, key) in enumerate(spec)]


A = ((32, 32, 32), "f32")
B = ((64, 64, 64), "f64")
C = ((128, 128, 128), "f32")


def test_every_request_completes_and_batches_form():
    clock = FakeClock()
    be = FakeBackend(clock)
    spec = [(0.0001 * i, A if i % 3 else B) for i in range(200)]
    stats = serve.Scheduler(be, budget_bytes=1 << 40, clock=clock).run(jobs_from(spec))
    assert stats.completed == 200 and stats.refused == 0 and stats.failed == 0
    assert max(stats.batch_hist) > 1                      # continuous batching merged requests
    assert all(len(r) <= be.max_batch for _, r, _ in be.launches)
    for key, rids, _ in be.launches:                     # a batch never mixes shapes
        assert all((spec[r][1] == key) for r in rids)
    assert be.max_live_streams <= be.num_streams
    assert stats.p99_ms >= stats.p50_ms > 0


def test_fifo_within_a_shape_and_no_starvation():
    """A steady stream of one shape cannot starve a request of another: the
    oldest waiting request's shape goes next whenever a stream frees."""
    clock = FakeClock()
    be = FakeBackend(clock, max_batch=2, num_streams=1)
    spec = [(0.0002 * i, A) for i in range(300)] + [(0.001, B)]
    stats = serve.Scheduler(be, budget_bytes=1 << 40, clock=clock).run(jobs_from(spec))
    assert stats.completed == 301
    order = [r for _, rids, _ in be.launches for r in rids]
    a_order = [r for r in order if r < 300]
    assert a_order == sorted(a_order)
    b_pos = order.index(300)
    # everything launched before B arrived before it (plus at most one batch in flight)
    assert all(spec[r][0] <= 0.001 + 1e-12 for r in order[:max(0, b_pos - 2)])
    assert b_pos < 40


def test_budget_is_never_exceeded_and_idle_executors_are_evicted():
    clock = FakeClock()
    be = FakeBackend(clock, num_streams=1, exec_bytes={A: 300 << 20, B: 300 << 20}, plan_bytes=10 << 20)
    budget = 700 << 20       # room for two plans and two executors at once
    spec = [(0.001 * i, A) for i in range(10)] + [(0.05 + 0.001 * i, B) for i in range(10)] + \
           [(0.1 + 0.001 * i, A) for i in range(10)]
    sch = serve.Scheduler(be, budget_bytes=budget, clock=clock)
    stats = sch.run(jobs_from(spec))
    assert stats.completed == 30
    assert stats.peak_bytes <= budget
    assert sch.used <= budget


def test_request_that_can_never_fit_is_refused():
    clock = FakeClock()
    be = FakeBackend(clock, exec_bytes={C: 10 << 30})
    spec = [(0.0, A), (0.0, C), (0.001, A)]
    stats = serve.Scheduler(be, budget_bytes=4 << 30, clock=clock).run(jobs_from(spec))
    assert stats.completed == 2 and stats.refused == 1


def test_waits_for_memory_instead_of_failing():
    """Two shapes whose executors cannot coexist: the second waits until the
    first's executor is idle, evicts it, and proceeds."""
    clock = FakeClock()
    be = FakeBackend(clock, num_streams=2, exec_bytes={A: 600 << 20, B: 600 << 20}, plan_bytes=1 << 20)
    spec = [(0.0, A)] * 3 + [(0.0, B)] * 3
    stats = serve.Scheduler(be, budget_bytes=700 << 20, clock=clock).run(jobs_from(spec))
    assert stats.completed == 6 and stats.evictions >= 1


def test_percentile():
    assert serve.percentile([1, 2, 3, 4], 0.5) == 2.5
    assert serve.percentile(list(range(101)), 0.99) == pytest.approx(99.0)


def test_prewarm_creates_idle_executors_within_budget():
    clock = FakeClock()
    be = FakeBackend(clock, exec_bytes={A: 300 << 20})
    sched = serve.Scheduler(be, budget_bytes=(1 << 20) + (700 << 20), clock=clock)
    assert sched.prewarm(A, 4) == 2                  # room for two executors after the plan
    assert be.created == [A, A] and sched.used <= sched.budget
    stats = sched.run(jobs_from([(0.0, A), (0.0, A)]))
    assert stats.completed == 2 and stats.executors_created == 0   # the run reused them


def test_backend_can_refuse_a_request():
    clock = FakeClock()
    be = FakeBackend(clock)
    be.accepts = lambda job: job.num_particles <= 500
    jobs = jobs_from([(0.0, A), (0.0, A)])
    jobs[1].num_particles = 400
    stats = serve.Scheduler(be, budget_bytes=1 << 40, clock=clock).run(jobs)
    assert stats.refused == 1 and stats.completed == 1 and jobs[0].status == "refused"


def test_busy_shape_batches_instead_of_growing_executors():
    """A burst of one shape with every executor of it busy: the waiting
    requests leave together when one comes back; no third executor is made."""
    clock = FakeClock()
    be = FakeBackend(clock, max_batch=8, num_streams=4)
    sched = serve.Scheduler(be, budget_bytes=8 << 30, clock=clock, max_per_key=2)
    jobs = jobs_from([(i * 2e-5, A) for i in range(20)])
    stats = sched.run(jobs)
    assert stats.completed == 20
    assert be.created.count(A) == 2
    assert max(len(r) for _, r, _ in be.launches) > 1
    # arrival order is kept within the shape
    order = [rid for _, r, _ in be.launches for rid in r]
    assert order == sorted(order)


class FaultyBackend(FakeBackend):
    """FakeBackend with injected failures: a launch that raises for one
    request, a completion that reports an error for another, and a launch
    whose completion stalls for `stall_s`."""

    def __init__(self, clock, raise_rid=None, error_rid=None, stall_rid=None, stall_s=0.0, **kw):
        super().__init__(clock, **kw)
        self.raise_rid, self.error_rid, self.stall_rid, self.stall_s = raise_rid, error_rid, stall_rid, stall_s
        self.errors = {}

    def launch(self, ex, jobs, stream):
        rids = [j.rid for j in jobs]
        if self.raise_rid in rids:
            raise RuntimeError("injected: launch failed")
        token = super().launch(ex, jobs, stream)
        if self.error_rid in rids:
            self.errors[token] = "injected: device error"
        if self.stall_rid in rids:
            self.inflight[token] += self.stall_s
        return token

    def error(self, token):
        return self.errors.pop(token, None)


def test_a_launch_that_raises_fails_only_its_batch():
    clock = FakeClock()
    be = FaultyBackend(clock, raise_rid=7, max_batch=1, num_streams=2)
    jobs = jobs_from([(0.0002 * i, A if i % 2 else B) for i in range(40)])
    sched = serve.Scheduler(be, budget_bytes=1 << 40, clock=clock)
    stats = sched.run(jobs)
    assert stats.failed == 1 and stats.completed == 39
    assert jobs[7].status == "failed" and "injected" in jobs[7].error
    assert all(j.status == "done" for j in jobs if j.rid != 7)
    # the failed executor was discarded and its bytes returned
    assert sched.used == sum(sched.plans.values()) + sum(
        len(v) * be.executor_bytes(k) for k, v in sched.idle.items())


def test_a_completion_with_an_error_fails_its_batch_and_discards_the_executor():
    clock = FakeClock()
    be = FaultyBackend(clock, error_rid=3, max_batch=4, num_streams=2)
    jobs = jobs_from([(0.0, A)] * 2 + [(0.001, A)] * 6)
    stats = serve.Scheduler(be, budget_bytes=1 << 40, clock=clock).run(jobs)
    bad = [j for j in jobs if j.status == "failed"]
    assert 3 in [j.rid for j in bad] and all(j.error == "injected: device error" for j in bad)
    assert stats.failed == len(bad) and stats.completed == 8 - len(bad)
    assert len(bad) <= be.max_batch
    assert A in be.destroyed


def test_a_stalled_batch_times_out_and_the_rest_proceeds():
    """One batch's completion stalls for 50 ms; with a 5 ms deadline its
    requests fail as timed out, requests of the same shape behind it use the
    other executor and stream, and the stalled executor is reused once the
    device finishes (its requests are not reported twice)."""
    clock = FakeClock()
    be = FaultyBackend(clock, stall_rid=2, stall_s=0.05, max_batch=1, num_streams=2)
    jobs = jobs_from([(0.0005 * i, A) for i in range(30)])
    sched = serve.Scheduler(be, budget_bytes=1 << 40, clock=clock, timeout_s=0.005)
    stats = sched.run(jobs)
    assert jobs[2].status == "timeout" and "running" in jobs[2].error
    assert stats.timed_out >= 1 and stats.completed + stats.timed_out == 30
    assert stats.failed == 0
    assert sum(1 for j in jobs if j.status == "done") == stats.completed
    assert be.created.count(A) <= 2 and not sched.busy and not sched.abandoned
    # the stalled batch's executor went back to the idle pool at the end
    assert len(sched.idle[A]) == be.created.count(A)


def test_requests_waiting_past_their_deadline_time_out():
    """One stream, slow solves and a burst: requests that cannot start before
    their deadline time out while waiting; those that do start complete."""
    clock = FakeClock()
    be = FakeBackend(clock, max_batch=1, num_streams=1)
    jobs = jobs_from([(0.0, C)] * 10)
    stats = serve.Scheduler(be, budget_bytes=1 << 40, clock=clock, timeout_s=0.006).run(jobs)
    late = [j for j in jobs if j.status == "timeout"]
    assert any("waiting" in j.error for j in late)
    assert all(("waiting" in j.error) or ("running" in j.error) for j in late)
    assert stats.completed + stats.timed_out == 10 and stats.completed >= 1
    assert all(j.done_s - j.arrival_s <= 0.006 + 0.005 for j in jobs if j.status == "done")
