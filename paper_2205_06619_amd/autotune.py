"""Autotuner of the fit kernel's launch shape.

The fit kernel's tiles are 64 x 64; what changes its speed on a given shape
is the speculative batch: how many trials the first batch of a row visit
evaluates (``batch_first``) and the largest batch (``batch_max``, which also
sizes the trial buffers), and for batched fits the number of workgroups
each fit runs on (``group_size``: the persistent launch is cut into groups
of that many workgroups, each taking fits from a queue).  None of them
changes a result (every fit is identical for any batch shape and group
size), so the tuner only times: for a shape bucket it runs a short prefix of
a fit (a few passes' worth of row visits) with each candidate and keeps the
fastest; for a batched workload it times the batched launch on a sample of
the problems, first over group sizes, then over batch shapes at the best
group size.  Choices are cached in a JSON file keyed by bucket, so a shape
is tuned once.

Buckets: the working shape (m' = min(m, n), n' = max(m, n)) and the rank,
each rounded up to a power of two.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

CANDIDATES: Tuple[Tuple[int, int], ...] = (
    (0, 0), (16, 0), (64, 0), (256, 0),
    (0, 256), (16, 256), (64, 256),
    (0, 1024), (64, 1024), (256, 1024),
)
GROUP_SIZES: Tuple[int, ...] = (1, 2, 4, 8, 16)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "stmf_autotune.json")


def _pow2(x: int) -> int:
    p = 1
    while p < x:
        p *= 2
    return p


def bucket(m: int, n: int, rank: int) -> str:
    mw, nw = min(m, n), max(m, n)
    return f"{_pow2(mw)}x{_pow2(nw)}r{_pow2(rank)}"


def choose(candidates: Iterable[Tuple[int, int]], timer: Callable[[int, int], float],
           repeats: int = 1) -> Tuple[Tuple[int, int], Dict[str, float]]:
    """The candidate with the smallest time (the first one on ties), and every
    candidate's best time over `repeats` runs."""
    times: Dict[str, float] = {}
    best, best_t = None, float("inf")
    for bf, bm in candidates:
        t = min(timer(bf, bm) for _ in range(repeats))
        times[f"{bf},{bm}"] = t
        if t < best_t:
            best, best_t = (bf, bm), t
    return best, times


class Cache:
    """JSON cache of tuned launch shapes: bucket -> {batch_first, batch_max,
    times}."""

    def __init__(self, path: Optional[str] = DEFAULT_CACHE):
        self.path = path
        self.data: Dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key: str) -> Optional[dict]:
        return self.data.get(key)

    def put(self, key: str, value: dict):
        self.data[key] = value
        if self.path:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def tune_fit(R, M, rank: int, passes: int = 2, seed: int = 0, cache: Optional[Cache] = None,
             candidates: Sequence[Tuple[int, int]] = CANDIDATES, visits: Optional[int] = None,
             **opts) -> dict:
    """Launch shape for one fit of this shape (device tensors R, M): each
    candidate runs the first `passes` passes' worth of row visits (or the
    first `visits` row visits: a short prefix keeps tuning a large matrix
    cheap); the kernel time decides.  Returns {batch_first, batch_max}
    (cached per bucket)."""
    from . import stmf
    m, n = R.shape
    key = "fit:" + bucket(m, n, rank)
    if cache is not None and cache.get(key):
        c = cache.get(key)
        return {"batch_first": c["batch_first"], "batch_max": c["batch_max"]}
    if visits is None:
        visits = passes * min(m, n)
    if visits < 1:
        raise ValueError("the tuning prefix needs at least one row visit")

    def timer(bf, bm):
        g = stmf.stmf_fit(R, M, rank, passes, seed=seed, batch_first=bf, batch_max=bm,
                          max_row_visits=visits, **opts)
        return g.info["kernel_ms"]

    (bf, bm), times = choose(candidates, timer)
    if cache is not None:
        cache.put(key, {"batch_first": bf, "batch_max": bm, "times_ms": times})
    return {"batch_first": bf, "batch_max": bm}


def sample_problems(problems: List[dict], sample: int) -> List[dict]:
    """`sample` problems spread over the population ordered by size (the
    largest, the smallest and evenly between), in that order."""
    order = sorted(problems, key=lambda p: -p["R"].numel())
    if sample >= len(order):
        return order
    step = (len(order) - 1) / max(sample - 1, 1)
    return [order[round(q * step)] for q in range(sample)]


def tune_batched(problems: List[dict], restarts: int = 1, sample: int = 16, iters: int = 2,
                 cache: Optional[Cache] = None, key: Optional[str] = None,
                 candidates: Sequence[Tuple[int, int]] = CANDIDATES,
                 group_sizes: Sequence[int] = GROUP_SIZES, visits: int = 0, **opts) -> dict:
    """Launch shape for a batched workload: the batched launch on `sample`
    problems spread over the population's sizes, with its restarts, for
    `iters` passes (or the first `visits` row visits of every fit: a prefix
    keeps tuning a population of large fits cheap); the wall time of the call
    decides, first among the group sizes (default batches), then among the
    batch shapes at the best group size.  Returns {group_size, batch_first,
    batch_max}."""
    import torch
    from . import stmf
    fields = ("group_size", "batch_first", "batch_max")
    if cache is not None and key and cache.get(key):
        c = cache.get(key)
        return {f: c[f] for f in fields}
    probe = [dict(p, iters=iters) for p in sample_problems(problems, sample)]

    def run(gs, bf, bm):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stmf.stmf_fit_batched(probe, restarts=restarts, group_size=gs, batch_first=bf,
                              batch_max=bm, max_row_visits=visits, **opts)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3

    run(group_sizes[0], 0, 0)  # first call pays the workspace allocation
    (gs, _), gtimes = choose([(g, 0) for g in group_sizes], lambda g, _: run(g, 0, 0))
    (bf, bm), times = choose(candidates, lambda bf, bm: run(gs, bf, bm))
    if cache is not None and key:
        cache.put(key, {"group_size": gs, "batch_first": bf, "batch_max": bm,
                        "group_times_ms": gtimes, "times_ms": times})
    return {"group_size": gs, "batch_first": bf, "batch_max": bm}
