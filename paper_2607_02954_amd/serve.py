"""Continuous-batching server for rollout jobs on one GPU.

Jobs (an initial world plus a step count) arrive over time.  Between chunks
of steps the server retires finished worlds and admits arrived jobs into free
slots while the device pool (the HBM budget) has room, so requests that
arrive while others run join the same persistent launches.  World state stays
resident on the device from admission to retirement.  Latency is measured from
arrival to retirement; the run reports p50/p99 latency and rollouts/s.

The scheduling logic is independent of the device: an executor supplies
admit/advance/remaining/retire, the clock is injectable, so the policy is
tested on the CPU with a fake executor and a virtual clock.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass
class JobResult:
    job_id: int
    arrival: float
    admitted: Optional[float]
    finished: Optional[float]
    steps: int
    ok: bool
    error: str = ""
    state: object = None

    @property
    def latency(self) -> float:
        return (self.finished - self.arrival) if self.finished is not None else float("nan")


class Unstable(RuntimeError):
    """A world was flagged (NaN or Mach guard) and has been evicted."""


class GpuExecutor:
    """Executor over a BatchEngine (device pool of world slots)."""

    def __init__(self, engine, params_for: Callable):
        self.engine = engine
        self.params_for = params_for
        self.capacity_slots = engine.max_worlds
        self.budget_bytes = engine.pool_bytes      # the library refuses what does not fit exactly

    def bytes_for(self, job) -> int:
        w = job.world
        return self.engine.world_bytes(self.params_for(job), w.n_filaments, w.n_particles)

    def admit(self, job) -> int:
        from .sim import SimError, SIM_E_FULL, SIM_E_WORKSPACE
        try:
            return self.engine.admit(job.world, self.params_for(job), job.steps)
        except SimError as e:
            if e.status in (SIM_E_FULL, SIM_E_WORKSPACE):
                raise MemoryError(str(e))
            raise

    def advance(self, n: int):
        self.engine.advance(n)

    def remaining(self, slot: int) -> int:
        return self.engine.remaining(slot)

    def retire(self, slot: int, job):
        from .sim import SimError, SIM_E_UNSTABLE
        try:
            return self.engine.retire(slot, job.world)
        except SimError as e:
            if e.status == SIM_E_UNSTABLE:
                raise Unstable(str(e))
            raise


@dataclass
class ServeStats:
    results: List[JobResult]
    makespan: float
    chunks: int
    peak_resident: int
    peak_bytes: int

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.results if r.ok])

    def summary(self) -> dict:
        lat = self.latencies()
        ok = int(sum(r.ok for r in self.results))
        return {
            "jobs": len(self.results), "completed": ok,
            "rollouts_per_s": ok / self.makespan if self.makespan > 0 else float("nan"),
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else float("nan"),
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else float("nan"),
            "makespan_s": self.makespan, "chunks": self.chunks,
            "peak_resident": self.peak_resident, "peak_bytes": self.peak_bytes,
        }


class Server:
    """First-fit continuous batching by slots and bytes.

    clock(): seconds since an arbitrary origin; wait(dt): block until dt
    seconds have passed (real sleep, or a virtual clock advance)."""

    def __init__(self, executor, chunk_steps: int = 20, clock: Callable[[], float] = time.perf_counter,
                 wait: Optional[Callable[[float], None]] = None, on_chunk: Optional[Callable] = None):
        if chunk_steps < 2 or chunk_steps % 2:
            raise ValueError("chunk_steps must be even and >= 2")
        self.ex = executor
        self.chunk = chunk_steps
        self.clock = clock
        self.wait = wait or (lambda dt: time.sleep(max(dt, 0.0)))
        self.on_chunk = on_chunk

    def run(self, jobs) -> ServeStats:
        ex = self.ex
        t0 = self.clock()
        now = lambda: self.clock() - t0
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        waiting: List = []                     # arrived, not yet admitted
        resident: Dict[int, tuple] = {}        # slot -> (job, bytes, admitted_at)
        results: Dict[int, JobResult] = {}
        used = 0
        chunks = peak_n = peak_b = 0
        while pending or waiting or resident:
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            # admission: first fit in arrival order
            still = []
            for job in waiting:
                need = ex.bytes_for(job)
                if need > ex.budget_bytes:
                    results[job.job_id] = JobResult(job.job_id, job.arrival, None, now(), job.steps, False,
                                                    "larger than the device budget")
                    continue
                if len(resident) < ex.capacity_slots and used + need <= ex.budget_bytes:
                    try:
                        slot = ex.admit(job)
                    except MemoryError:
                        still.append(job)
                        continue
                    used += need
                    resident[slot] = (job, need, now())
                else:
                    still.append(job)
            waiting = still
            peak_n = max(peak_n, len(resident))
            peak_b = max(peak_b, used)
            if not resident:
                if pending:
                    self.wait(pending[0].arrival - now())
                    continue
                if waiting:   # nothing fits and nothing runs: cannot make progress
                    for job in waiting:
                        results[job.job_id] = JobResult(job.job_id, job.arrival, None, now(), job.steps, False,
                                                        "could not be admitted")
                    waiting = []
                continue
            ex.advance(self.chunk)
            chunks += 1
            if self.on_chunk:
                self.on_chunk(self, resident)
            for slot in [s for s in resident if ex.remaining(s) == 0]:
                job, need, adm = resident.pop(slot)
                used -= need
                try:
                    state = ex.retire(slot, job)
                    results[job.job_id] = JobResult(job.job_id, job.arrival, adm, now(), job.steps, True, state=state)
                except Unstable as e:
                    results[job.job_id] = JobResult(job.job_id, job.arrival, adm, now(), job.steps, False, str(e))
        ordered = [results[j.job_id] for j in sorted(jobs, key=lambda j: j.job_id)]
        return ServeStats(ordered, now(), chunks, peak_n, peak_b)
