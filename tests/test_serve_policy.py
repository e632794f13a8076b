"""Continuous-batching policy on the CPU: a fake executor and a virtual clock."""
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
