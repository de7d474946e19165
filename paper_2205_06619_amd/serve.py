"""Continuous-batching serving loop over the FastSTMF engine.

Completion jobs (a masked matrix R, its rank, passes and seed) arrive over
time.  Each tick of the loop:

  1. moves the jobs whose arrival time has passed into a FIFO wait queue;
  2. admits waiting jobs, oldest first, while the engine has a free slot and
     arena room for the job's footprint (``stmf_engine_job_footprint``): R,
     the mask, the factors and the fit state stay resident in device memory
     from admission to retirement;
  3. advances every resident job by at most ``rows_per_tick`` row visits
     (``stmf_batch_tick``: each job on a group of workgroups, by default as
     many as it has 64 x 64 tiles, the jobs side by side over the device, so
     jobs that arrived while others were running share it with them);
  4. retires the jobs that finished and records their latency (finish time
     minus arrival time).

Every job's result is the one ``stmf_fit`` gives alone with the job's group
size and the same seed (with the default group size, ``stmf_fit``'s own
result): a job's arithmetic never depends on which other jobs share its
launches.  ``sequential`` runs the same stream through the plain
one-fit-at-a-time path for comparison.

The device calls go through a small backend object so that the queueing and
bookkeeping can be exercised without a GPU (``EngineBackend`` is the real
one).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclass
class Job:
    jid: int
    arrival: float          # seconds after the start of the run
    R: object               # device tensor, float32 m x n
    M: object               # device tensor, uint8 m x n
    rank: int
    iters: int
    seed: int
    admitted: float = math.nan
    finished: float = math.nan
    result: object = None

    @property
    def shape(self):
        return tuple(self.R.shape)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeStats:
    jobs: int
    wall_s: float
    jobs_per_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    ticks: int = 0
    max_resident: int = 0
    latencies_ms: List[float] = field(default_factory=list)

    def as_dict(self):
        d = dict(self.__dict__)
        d.pop("latencies_ms")
        return d


def percentile(values: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    xs = sorted(values)
    if not xs:
        raise ValueError("percentile of an empty sequence")
    rank = max(1, math.ceil(q / 100.0 * len(xs)))
    return xs[min(rank, len(xs)) - 1]


def summarize(jobs: Sequence[Job], wall_s: float, ticks: int = 0, max_resident: int = 0) -> ServeStats:
    lat = [j.latency * 1e3 for j in jobs]
    return ServeStats(jobs=len(jobs), wall_s=wall_s, jobs_per_s=len(jobs) / wall_s if wall_s > 0 else 0.0,
                      p50_ms=percentile(lat, 50), p99_ms=percentile(lat, 99),
                      mean_ms=float(np.mean(lat)), ticks=ticks, max_resident=max_resident,
                      latencies_ms=lat)


class EngineBackend:
    """The engine's C entry points (through the Python binding)."""

    def __init__(self, arena_bytes: int, max_slots: int, opt=None, stream=None, **kw):
        from . import stmf
        self.S = stmf
        self.stream = stream
        self.eng = stmf.stmf_engine_create(arena_bytes, max_slots, opt, **kw)
        self.capacity = arena_bytes

    def footprint(self, job: Job) -> int:
        m, n = job.shape
        return self.S.stmf_engine_job_footprint(self.eng, m, n, job.rank, job.iters)

    def admit(self, job: Job) -> Optional[int]:
        return self.S.stmf_engine_admit(self.eng, job.R, job.M, job.rank, job.iters, job.seed,
                                        stream=self.stream)

    def tick(self, rows: int):
        self.S.stmf_batch_tick(self.eng, rows, stream=self.stream)

    def poll(self, slot: int) -> bool:
        return self.S.stmf_engine_poll(self.eng, slot, stream=self.stream)

    def retire(self, slot: int):
        return self.S.stmf_engine_retire(self.eng, slot, stream=self.stream)

    def close(self):
        self.S.stmf_engine_destroy(self.eng)


class Server:
    """The continuous-batching loop (see the module docstring)."""

    def __init__(self, backend, rows_per_tick: int = 8,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        if rows_per_tick < 1:
            raise ValueError("rows_per_tick must be at least 1")
        self.backend = backend
        self.rows_per_tick = rows_per_tick
        self.clock = clock
        self.sleep = sleep

    def run(self, jobs: Sequence[Job]) -> ServeStats:
        for j in jobs:
            if self.backend.footprint(j) > self.backend.capacity:
                raise ValueError(f"job {j.jid} needs {self.backend.footprint(j)} bytes, more than "
                                 f"the arena's {self.backend.capacity}")
        pending = deque(sorted(jobs, key=lambda j: (j.arrival, j.jid)))
        waiting: deque = deque()
        resident = {}
        ticks = max_res = 0
        t0 = self.clock()
        while pending or waiting or resident:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:
                slot = self.backend.admit(waiting[0])
                if slot is None:
                    break  # no slot or no arena room: wait for a retirement
                job = waiting.popleft()
                job.admitted = self.clock() - t0
                resident[slot] = job
            max_res = max(max_res, len(resident))
            if not resident:
                if waiting:
                    raise RuntimeError("a waiting job cannot be admitted into an empty engine")
                self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                continue
            self.backend.tick(self.rows_per_tick)
            ticks += 1
            for slot in list(resident):
                if self.backend.poll(slot):
                    job = resident.pop(slot)
                    job.result = self.backend.retire(slot)
                    job.finished = self.clock() - t0
        wall = self.clock() - t0
        return summarize(jobs, wall, ticks, max_res)


def sequential(jobs: Sequence[Job], fit: Callable[[Job], object],
               clock: Callable[[], float] = time.perf_counter,
               sleep: Callable[[float], None] = time.sleep) -> ServeStats:
    """The plain path: one fit at a time in arrival order, each starting when
    it has arrived and the previous one has finished."""
    t0 = clock()
    for job in sorted(jobs, key=lambda j: (j.arrival, j.jid)):
        now = clock() - t0
        if job.arrival > now:
            sleep(job.arrival - now)
        job.admitted = clock() - t0
        job.result = fit(job)
        job.finished = clock() - t0
    return summarize(jobs, clock() - t0)


def synthetic_jobs(count: int, rate_per_s: float, seed: int = 5, m_range=(50, 1000),
                   n_range=(50, 5000), r_range=(2, 30), miss_range=(0.2, 0.8), iters: int = 30,
                   device="cuda") -> List[Job]:
    """A Poisson stream of FP32 noisy planted completion jobs, sized as the
    batched workload (shape, rank and missing fraction drawn uniformly)."""
    import torch
    from . import synth
    probs = synth.batched_problems(count, seed=seed, integer=False, m_range=m_range,
                                   n_range=n_range, r_range=r_range, miss_range=miss_range)
    arrivals = synth.poisson_arrivals(count, rate_per_s, seed=seed)
    jobs = []
    for p, t in zip(probs, arrivals):
        jobs.append(Job(jid=p.pid, arrival=float(t), R=torch.from_numpy(p.R).to(device),
                        M=torch.from_numpy(p.M).to(device), rank=p.rank, iters=iters,
                        seed=1000 + p.pid))
    return jobs
