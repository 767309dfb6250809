"""Continuous-batching request loop over the pool API (md_pool_*).

Jobs (independent simulations) arrive over time.  The loop admits waiting jobs
in arrival order while the pool has device memory and a free slot
(md_pool_admit returns MD_EAGAIN otherwise), advances every resident job
together by one chunk of steps (md_pool_launch, which returns while the chunk
runs, so the next admissions overlap it; md_pool_poll collects it), and
fetches and releases the jobs that finished, so later arrivals are admitted as
soon as room frees up and their work shares launches with the jobs already
running; the finished jobs of a chunk are fetched together (md_pool_fetch_many).
Latency of a job is its completion time minus its arrival time.

`run_plain` is the reference point: one job at a time, one context per job,
one launch per step (no graphs), the same kernels.
"""
from __future__ import annotations

import collections
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import md


@dataclass
class Job:
    jid: int
    arrival: float            # seconds after the stream starts
    params: md.Params
    surface: str
    surf: tuple
    x: np.ndarray
    p: np.ndarray
    nsteps: int
    admitted: float | None = None
    finished: float | None = None
    status: int | None = None
    result: dict | None = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def serve(jobs, budget_bytes: int, max_jobs: int, chunk: int = 32, realtime: bool = True,
          keep_results: bool = False, pool_factory=None, clock=time.perf_counter, sleep=time.sleep):
    """Run `jobs` through one pool; returns (jobs, pool stats).  With
    realtime=False every job counts as arrived at t = 0 (closed loop).

    Each round enqueues one chunk for the resident jobs (md_pool_launch) and,
    while it runs, admits the jobs that are waiting; then it collects the
    chunk (md_pool_poll) and fetches and releases the jobs it finished."""
    make = pool_factory or (lambda: md.Pool(budget_bytes, max_jobs))
    if not realtime:
        for j in jobs:
            j.arrival = 0.0  # closed loop: every job is waiting at t = 0
    pool = make()
    pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    waiting = collections.deque()
    resident = {}
    running = False  # a chunk is in flight
    t0 = clock()
    try:
        while pending or waiting or resident:
            now = clock() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            while waiting:
                j = waiting[0]
                pid = pool.admit(j.params, j.surface, j.surf, j.x, j.p, j.nsteps)
                if pid is None:
                    break
                j.admitted = clock() - t0
                resident[pid] = j
                waiting.popleft()
            freed = False
            if running:
                done = pool.poll()
                # the finished jobs' states, read together (one wait)
                for pid, (rc, res) in zip(done, pool.fetch_many(done)):
                    j = resident.pop(pid)
                    j.finished = clock() - t0
                    j.status = rc
                    if keep_results:
                        j.result = res
                    pool.release(pid)
                    freed = True
                running = False
            if resident:
                pool.launch(chunk)
                running = True
            elif freed:
                continue  # room for the waiting jobs
            elif pending and realtime:
                sleep(max(0.0, pending[0].arrival - (clock() - t0)))
            elif waiting:
                raise RuntimeError(f"job {waiting[0].jid} does not fit an empty pool")
        stats = pool.stats()
    finally:
        pool.close()
    return jobs, stats


def run_plain(jobs, realtime: bool = True, keep_results: bool = False, clock=time.perf_counter,
              sleep=time.sleep):
    """One job at a time, per-step launches without graphs."""
    if not realtime:
        for j in jobs:
            j.arrival = 0.0
    prev = os.environ.get("MD_NO_GRAPH")
    os.environ["MD_NO_GRAPH"] = "1"
    t0 = clock()
    try:
        for j in sorted(jobs, key=lambda q: q.arrival):
            if realtime:
                sleep(max(0.0, j.arrival - (clock() - t0)))
            j.admitted = clock() - t0
            s = md.System(j.params, j.surface, j.surf)
            s.set_particles(j.x, j.p)
            s.step(j.nsteps)
            st = s.get_state(want_force=False)
            s.close()
            j.finished = clock() - t0
            j.status = 0
            if keep_results:
                j.result = st
    finally:
        if prev is None:
            os.environ.pop("MD_NO_GRAPH", None)
        else:
            os.environ["MD_NO_GRAPH"] = prev
    return jobs


def summarize(jobs, wall: float | None = None) -> dict:
    lat = np.array([j.latency for j in jobs if j.finished is not None])
    span = wall if wall is not None else max(j.finished for j in jobs) - min(j.arrival for j in jobs)
    ps = sum(j.n * j.nsteps for j in jobs)
    return {
        "jobs": len(jobs),
        "jobs_per_s": len(jobs) / span,
        "particle_steps_per_s": ps / span,
        "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
        "max_latency_s": float(lat.max()) if lat.size else None,
        "failed": sum(1 for j in jobs if j.status not in (0, None)),
    }
