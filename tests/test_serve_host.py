"""Host logic of the serving loop (queueing, admission, latency bookkeeping)
with a fake backend and a virtual clock: no GPU."""
import numpy as np
import pytest

from paper_2205_06619_amd import serve


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeBackend:
    """Slots with a byte budget; a job finishes after `work` ticks, each tick
    taking `tick_s` of virtual time."""

    def __init__(self, clock, capacity, max_slots, tick_s=1.0):
        self.clock, self.capacity, self.max_slots, self.tick_s = clock, capacity, max_slots, tick_s
        self.res = {}
        self.used = 0
        self.admit_log = []

    def footprint(self, job):
        return job.R.size

    def admit(self, job):
        if len(self.res) >= self.max_slots or self.used + self.footprint(job) > self.capacity:
            return None
        slot = next(s for s in range(self.max_slots) if s not in self.res)
        self.res[slot] = [job, job.iters]
        self.used += self.footprint(job)
        self.admit_log.append((job.jid, self.clock()))
        return slot

    def tick(self, rows):
        self.clock.t += self.tick_s
        for v in self.res.values():
            v[1] -= 1

    def poll(self, slot):
        return self.res[slot][1] <= 0

    def retire(self, slot):
        job, _ = self.res.pop(slot)
        self.used -= self.footprint(job)
        return ("result", job.jid)


def _job(jid, arrival, size, work):
    return serve.Job(jid=jid, arrival=arrival, R=np.zeros(size, np.float32),
                     M=np.zeros(size, np.uint8), rank=2, iters=work, seed=jid)


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert serve.percentile(xs, 50) == 50
    assert serve.percentile(xs, 99) == 99
    assert serve.percentile(xs, 100) == 100
    assert serve.percentile([7.0], 99) == 7.0
    assert serve.percentile([3, 1, 2], 50) == 2
    with pytest.raises(ValueError):
        serve.percentile([], 50)


def test_fifo_admission_by_footprint():
    clk = VClock()
    be = FakeBackend(clk, capacity=100, max_slots=8)
    # each job needs 60% of the arena: one resident at a time, in arrival order
    jobs = [_job(0, 0.0, 60, 3), _job(1, 0.5, 60, 2), _job(2, 0.6, 60, 1)]
    st = serve.Server(be, rows_per_tick=1, clock=clk, sleep=clk.sleep).run(jobs)
    assert [j for j, _ in be.admit_log] == [0, 1, 2]
    assert st.max_resident == 1
    assert [jb.result for jb in jobs] == [("result", 0), ("result", 1), ("result", 2)]
    # job 0: ticks 1..3 -> done at 3; job 1 admitted at 3, done at 5; job 2 at 6
    assert [jb.finished for jb in jobs] == [3.0, 5.0, 6.0]
    assert [round(jb.latency, 6) for jb in jobs] == [3.0, 4.5, 5.4]
    assert st.jobs == 3 and st.ticks == 6


def test_continuous_batching_admits_while_others_run():
    clk = VClock()
    be = FakeBackend(clk, capacity=1000, max_slots=4)
    jobs = [_job(0, 0.0, 10, 10), _job(1, 2.5, 10, 2), _job(2, 2.6, 10, 2)]
    st = serve.Server(be, rows_per_tick=1, clock=clk, sleep=clk.sleep).run(jobs)
    # jobs 1 and 2 join job 0 at the first tick after they arrive (t = 3)
    assert dict(be.admit_log) == {0: 0.0, 1: 3.0, 2: 3.0}
    assert st.max_resident == 3
    assert jobs[1].finished == 5.0 and jobs[2].finished == 5.0 and jobs[0].finished == 10.0
    assert st.p50_ms == pytest.approx(2.5e3) and st.p99_ms == pytest.approx(10e3)


def test_slot_limit_and_idle_gaps():
    clk = VClock()
    be = FakeBackend(clk, capacity=10 ** 6, max_slots=1)
    jobs = [_job(0, 5.0, 1, 1), _job(1, 5.0, 1, 1), _job(2, 20.0, 1, 2)]
    st = serve.Server(be, rows_per_tick=1, clock=clk, sleep=clk.sleep).run(jobs)
    assert [jb.finished for jb in jobs] == [6.0, 7.0, 22.0]
    assert st.max_resident == 1
    assert st.wall_s == 22.0


def test_job_larger_than_arena_is_rejected():
    clk = VClock()
    be = FakeBackend(clk, capacity=50, max_slots=2)
    with pytest.raises(ValueError):
        serve.Server(be, clock=clk, sleep=clk.sleep).run([_job(0, 0.0, 51, 1)])


def test_sequential_plain_path():
    clk = VClock()

    def fit(job):
        clk.t += job.iters
        return job.jid

    jobs = [_job(0, 1.0, 1, 2), _job(1, 1.5, 1, 3), _job(2, 10.0, 1, 1)]
    st = serve.sequential(jobs, fit, clock=clk, sleep=clk.sleep)
    assert [jb.finished for jb in jobs] == [3.0, 6.0, 11.0]
    assert [jb.result for jb in jobs] == [0, 1, 2]
    assert st.jobs_per_s == pytest.approx(3 / 11.0)
