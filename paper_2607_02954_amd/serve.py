"""Continuous-batching server for rollout jobs on one GPU.

Jobs (an initial world plus a step count) arrive over time.  Between chunks
of steps the server retires finished worlds and admits arrived jobs into free
slots while the device pool (the HBM budget) has room, so requests that
arrive while others run join the same persistent launches.  World state stays
resident on the device from admission to retirement.  Latency is measured from
arrival to retirement; the run reports p50/p99 latency and rollouts/s.

Jobs come from a fixed arrival trace (run) or are submitted live, from
producer threads or asyncio, while the loop runs (submit / serve): the
evolutionary-search workers of the paper's controller experiments submit
candidate rollouts this way.

The scheduling logic is independent of the device: an executor supplies
admit/advance/remaining/retire, the clock is injectable, so the policy is
tested on the CPU with a fake executor and a virtual clock.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from concurrent.futures import Future
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

    Jobs reach the loop in two ways: a pre-built arrival trace (run(jobs):
    job.arrival seconds after the start) and live submission (submit(job),
    thread-safe, from producer threads or, through submit_async, an asyncio
    loop) while serve() runs.  A live job arrives when it is submitted.  All
    device work happens on the thread that runs the loop.

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
        self._cv = threading.Condition()
        self._inbox: deque = deque()           # (job, future, submitted at), under _cv
        self._closed = False

    # -- live submission -------------------------------------------------
    def submit(self, job) -> Future:
        """Queue a job while the loop runs; the future resolves to its
        JobResult when it retires (or is rejected).  Thread-safe."""
        fut: Future = Future()
        with self._cv:
            if self._closed:
                raise RuntimeError("server is closed to new jobs")
            self._inbox.append((job, fut, self.clock()))
            self._cv.notify()
        return fut

    async def submit_async(self, job) -> JobResult:
        """submit() for asyncio producers: await the job's JobResult."""
        import asyncio
        return await asyncio.wrap_future(self.submit(job))

    def close(self):
        """No further submissions; serve() returns once every job has retired."""
        with self._cv:
            self._closed = True
            self._cv.notify()

    def serve(self, idle_poll: float = 0.05) -> ServeStats:
        """Run the loop on submitted jobs until close() and the queue drains.
        Results are listed in submission order."""
        return self._loop([], live=True, idle_poll=idle_poll)

    def run(self, jobs) -> ServeStats:
        """Run a fixed arrival trace to completion (results in job_id order)."""
        return self._loop(jobs, live=False)

    # -- the loop --------------------------------------------------------
    def _loop(self, jobs, live: bool, idle_poll: float = 0.05) -> ServeStats:
        ex = self.ex
        t0 = self.clock()
        now = lambda: self.clock() - t0
        # every job gets a key: trace jobs in job_id order, live jobs in
        # submission order after them; results are listed by key
        trace = sorted(jobs, key=lambda j: j.job_id)
        key_of = {id(j): k for k, j in enumerate(trace)}
        n_keys = len(trace)
        pending = deque(sorted(trace, key=lambda j: j.arrival))
        waiting: List = []                     # (key, job, arrival, future): arrived, not admitted
        resident: Dict[int, tuple] = {}        # slot -> (key, job, bytes, admitted_at, arrival, future)
        results: Dict[int, JobResult] = {}
        used = 0
        chunks = peak_n = peak_b = 0

        def finish(key, fut, res):
            results[key] = res
            if fut is not None:
                fut.set_result(res)

        def take_inbox(block: bool) -> bool:
            """Move submitted jobs to the waiting list; True once the server is
            closed and nothing more can arrive."""
            nonlocal n_keys
            with self._cv:
                if block and not self._inbox and not self._closed:
                    self._cv.wait(idle_poll)
                while self._inbox:
                    job, fut, sub = self._inbox.popleft()
                    waiting.append((n_keys, job, sub - t0, fut))
                    n_keys += 1
                return self._closed and not self._inbox

        while True:
            drained = take_inbox(False) if live else True
            t = now()
            while pending and pending[0].arrival <= t:
                j = pending.popleft()
                waiting.append((key_of[id(j)], j, j.arrival, None))
            if drained and not pending and not waiting and not resident:
                break
            # admission: first fit in arrival order
            still = []
            for key, job, arr, fut in waiting:
                need = ex.bytes_for(job)
                if need > ex.budget_bytes:
                    finish(key, fut, JobResult(job.job_id, arr, None, now(), job.steps, False,
                                               "larger than the device budget"))
                    continue
                if len(resident) < ex.capacity_slots and used + need <= ex.budget_bytes:
                    try:
                        slot = ex.admit(job)
                    except MemoryError:
                        still.append((key, job, arr, fut))
                        continue
                    used += need
                    resident[slot] = (key, job, need, now(), arr, fut)
                else:
                    still.append((key, job, arr, fut))
            waiting = still
            peak_n = max(peak_n, len(resident))
            peak_b = max(peak_b, used)
            if not resident:
                if waiting:
                    # nothing fits an idle device: no retirement can free room
                    for key, job, arr, fut in waiting:
                        finish(key, fut, JobResult(job.job_id, arr, None, now(), job.steps, False,
                                                   "could not be admitted"))
                    waiting = []
                    continue
                if pending:
                    self.wait(pending[0].arrival - now())
                    continue
                if live and not drained:
                    take_inbox(True)           # idle: sleep until a submission (or a poll tick)
                continue
            ex.advance(self.chunk)
            chunks += 1
            if self.on_chunk:
                self.on_chunk(self, resident)
            for slot in [s for s in resident if ex.remaining(s) == 0]:
                key, job, need, adm, arr, fut = resident.pop(slot)
                used -= need
                try:
                    state = ex.retire(slot, job)
                    res = JobResult(job.job_id, arr, adm, now(), job.steps, True, state=state)
                except Unstable as e:
                    res = JobResult(job.job_id, arr, adm, now(), job.steps, False, str(e))
                finish(key, fut, res)
        ordered = [results[k] for k in range(n_keys)]
        return ServeStats(ordered, now(), chunks, peak_n, peak_b)
