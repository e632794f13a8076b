"""Continuous-batching policy on the CPU: a fake executor and a virtual clock."""
import time
from dataclasses import dataclass

import pytest

from paper_2607_02954_amd.serve import Server, Unstable


@dataclass
class FakeJob:
    job_id: int
    arrival: float
    steps: int
    nbytes: int
    unstable: bool = False


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def wait(self, dt):
        self.t += max(dt, 0.0)


class FakeExecutor:
    """Tracks steps per slot; every chunk costs `step_cost` virtual seconds per step."""

    def __init__(self, clock, slots=4, budget=100, step_cost=1e-3):
        self.clock, self.capacity_slots, self.budget_bytes, self.step_cost = clock, slots, budget, step_cost
        self.rem, self.jobs, self.log = {}, {}, []
        self.steps_run = {}

    def bytes_for(self, job):
        return job.nbytes

    def admit(self, job):
        free = [s for s in range(self.capacity_slots) if s not in self.rem]
        assert free, "server admitted beyond the slot capacity"
        used = sum(self.jobs[s].nbytes for s in self.rem)
        assert used + job.nbytes <= self.budget_bytes, "server admitted beyond the budget"
        s = free[0]
        self.rem[s], self.jobs[s] = job.steps, job
        self.steps_run[job.job_id] = 0
        self.log.append(("admit", job.job_id, self.clock()))
        return s

    def advance(self, n):
        for s in self.rem:
            ran = min(self.rem[s], n)
            self.rem[s] -= ran
            self.steps_run[self.jobs[s].job_id] += ran
        self.clock.t += n * self.step_cost

    def remaining(self, s):
        return self.rem[s]

    def retire(self, s, job):
        del self.rem[s]
        del self.jobs[s]
        self.log.append(("retire", job.job_id, self.clock()))
        if job.unstable:
            raise Unstable("flagged")
        return "state-%d" % job.job_id


def test_admission_respects_slots_and_budget_and_runs_exact_steps():
    clk = Clock()
    ex = FakeExecutor(clk, slots=3, budget=100)
    jobs = [FakeJob(i, 0.01 * i, 30 + 17 * i, 40 if i % 2 else 25) for i in range(10)]
    st = Server(ex, chunk_steps=10, clock=clk, wait=clk.wait).run(jobs)
    assert all(r.ok for r in st.results)
    for j in jobs:
        assert ex.steps_run[j.job_id] == j.steps           # never more, never fewer
    assert st.peak_resident <= 3 and st.peak_bytes <= 100
    for r in st.results:
        assert r.admitted >= r.arrival and r.finished >= r.admitted


def test_late_arrivals_join_running_batch():
    clk = Clock()
    ex = FakeExecutor(clk, slots=4, budget=100, step_cost=1e-3)
    long_job = FakeJob(0, 0.0, 1000, 10)
    late = FakeJob(1, 0.1, 20, 10)                      # arrives while job 0 runs
    st = Server(ex, chunk_steps=10, clock=clk, wait=clk.wait).run([long_job, late])
    r0, r1 = st.results
    assert r1.admitted < r0.finished                    # overlapped, not queued behind
    assert r1.finished < r0.finished


def test_slot_reuse_and_fcfs_first_fit():
    clk = Clock()
    ex = FakeExecutor(clk, slots=1, budget=100)
    jobs = [FakeJob(i, 0.0, 10, 10) for i in range(5)]
    st = Server(ex, chunk_steps=10, clock=clk, wait=clk.wait).run(jobs)
    order = [jid for kind, jid, _ in ex.log if kind == "admit"]
    assert order == [0, 1, 2, 3, 4] and st.chunks == 5


def test_unstable_world_is_evicted_without_affecting_others():
    clk = Clock()
    ex = FakeExecutor(clk, slots=4, budget=100)
    jobs = [FakeJob(0, 0.0, 40, 10), FakeJob(1, 0.0, 40, 10, unstable=True), FakeJob(2, 0.0, 60, 10)]
    st = Server(ex, chunk_steps=10, clock=clk, wait=clk.wait).run(jobs)
    assert [r.ok for r in st.results] == [True, False, True]
    assert ex.steps_run[0] == 40 and ex.steps_run[2] == 60


def test_oversized_job_is_rejected_and_idle_waits_for_arrivals():
    clk = Clock()
    ex = FakeExecutor(clk, slots=2, budget=50)
    jobs = [FakeJob(0, 5.0, 10, 60), FakeJob(1, 7.0, 10, 10)]
    st = Server(ex, chunk_steps=10, clock=clk, wait=clk.wait).run(jobs)
    assert not st.results[0].ok and "budget" in st.results[0].error
    assert st.results[1].ok and st.results[1].admitted >= 7.0
    s = st.summary()
    assert s["completed"] == 1 and s["p99_latency_s"] >= s["p50_latency_s"]


def test_chunk_must_be_even():
    with pytest.raises(ValueError):
        Server(FakeExecutor(Clock()), chunk_steps=7)


def test_live_submissions_join_the_running_batch():
    """Jobs submitted while the loop runs (here from the chunk callback, on
    the virtual clock) are admitted between chunks beside the running ones."""
    clk = Clock()
    ex = FakeExecutor(clk, slots=4, budget=100, step_cost=1e-3)
    futures = {}
    schedule = {2: 1, 4: 2, 6: 3}                    # chunk number -> job submitted after it
    seen = {"chunks": 0}

    def producer(srv, resident):
        seen["chunks"] += 1
        k = schedule.get(seen["chunks"])
        if k is not None:
            futures[k] = srv.submit(FakeJob(k, None, 30 + 10 * k, 20))
            if k == 3:
                srv.close()

    srv = Server(ex, chunk_steps=10, clock=clk, wait=clk.wait, on_chunk=producer)
    futures[0] = srv.submit(FakeJob(0, None, 200, 30))
    st = srv.serve()
    assert len(st.results) == 4 and all(r.ok for r in st.results)
    assert [r.job_id for r in st.results] == [0, 1, 2, 3]          # submission order
    for k, fut in futures.items():
        assert fut.done() and fut.result().ok
        assert ex.steps_run[k] == fut.result().steps                # exact step counts
    r0 = futures[0].result()
    for k in (1, 2, 3):
        rk = futures[k].result()
        assert rk.arrival > 0 and rk.admitted < r0.finished         # joined while job 0 ran
        assert rk.admitted - rk.arrival <= 10 * ex.step_cost + 1e-12   # within one chunk


class SleepyExecutor(FakeExecutor):
    """Fake executor on the real clock: every chunk sleeps briefly."""

    def advance(self, n):
        for s in self.rem:
            ran = min(self.rem[s], n)
            self.rem[s] -= ran
            self.steps_run[self.jobs[s].job_id] += ran
        time.sleep(n * self.step_cost)


def test_submissions_from_producer_threads():
    import threading
    clk = time.perf_counter
    ex = SleepyExecutor(clk, slots=3, budget=100, step_cost=2e-4)
    srv = Server(ex, chunk_steps=10)
    futs, lock = [], threading.Lock()

    def producer(base):
        for i in range(6):
            f = srv.submit(FakeJob(base + i, None, 20 + 10 * i, 20 + (i % 3) * 10))
            with lock:
                futs.append((base + i, f))
            time.sleep(0.003)

    threads = [threading.Thread(target=producer, args=(100 * k,)) for k in range(3)]
    for t in threads:
        t.start()
    closer = threading.Thread(target=lambda: ([t.join() for t in threads], srv.close()))
    closer.start()
    st = srv.serve(idle_poll=0.005)
    closer.join()
    assert len(st.results) == 18 and all(r.ok for r in st.results)
    for jid, f in futs:
        r = f.result(timeout=1)
        assert r.ok and r.job_id == jid and ex.steps_run[jid] == r.steps
        assert r.finished >= r.admitted >= r.arrival
    assert st.peak_resident <= 3 and st.peak_bytes <= 100
    with pytest.raises(RuntimeError):
        srv.submit(FakeJob(999, None, 10, 10))                      # closed


def test_asyncio_producer():
    import asyncio
    import threading
    ex = SleepyExecutor(time.perf_counter, slots=2, budget=100, step_cost=1e-4)
    srv = Server(ex, chunk_steps=10)
    out = {}

    async def produce():
        tasks = []
        for i in range(5):
            tasks.append(asyncio.ensure_future(srv.submit_async(FakeJob(i, None, 20 + 5 * i, 30))))
            await asyncio.sleep(0.002)
        out["res"] = await asyncio.gather(*tasks)
        srv.close()

    th = threading.Thread(target=lambda: asyncio.run(produce()))
    th.start()
    st = srv.serve(idle_poll=0.005)
    th.join()
    assert [r.job_id for r in out["res"]] == [0, 1, 2, 3, 4]
    assert all(r.ok for r in out["res"]) and len(st.results) == 5
