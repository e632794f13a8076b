"""Batched worlds and the continuous-batching server on the GPU.

Each world's result in a batch (and in the served mix) must equal the same
world run alone through sim_rollout: bitwise with the binned transfer, whose
sums are order-independent 64-bit fixed point.  Each retired world is also
compared with the FP64 oracle run from its initial state for the same steps:
positions (e_x <= 1e-5), the last step's grid velocity (e_u <= 1e-4) and the
displacement over the run (e_d <= 1e-4); errors are printed.
"""
import time

import numpy as np
import pytest
import torch

from paper_2607_02954_amd import workloads as wl
from parity_util import TOL_D, TOL_U, TOL_X, final_state_errors, oracle_params

pytestmark = pytest.mark.gpu


def _mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_02954_amd import sim, batch, serve
    return sim, batch, serve


def _alone(sim, w, steps, **kw):
    W = sim.World(w, sim.Params(nx=w.nx, ny=w.ny, **kw))
    W.rollout(0, steps)
    torch.cuda.synchronize()
    return W.state


def _same(a, b):
    return (torch.equal(a.cell.cpu(), b.cell.cpu()) and torch.equal(a.frac.cpu(), b.frac.cpu())
            and torch.equal(a.f.cpu(), b.f.cpu()) and torch.equal(a.u.cpu(), b.u.cpu()))


def _worlds():
    return [wl.random_world(10 + i, nx, ny, lens, amp=0.5)
            for i, (nx, ny, lens) in enumerate([(64, 64, [20, 9]), (96, 64, [40] * 6), (128, 128, [64] * 20),
                                                (72, 50, [3, 1, 17]), (64, 96, [12] * 30)])]


def _check_oracle(sim, w, st, steps, label):
    op = oracle_params(sim.Params(nx=w.nx, ny=w.ny))
    ex, ea, eu, ed = final_state_errors(w, st, op, 0, steps)
    print(f"{label}, {steps} steps vs oracle: e_x={ex:.2e} e_a={ea:.2e} cells e_u={eu:.2e} e_d={ed:.2e}")
    assert ex <= TOL_X and eu <= TOL_U and ed <= TOL_D, (label, ex, eu, ed)


def test_batch_equals_single_worlds():
    sim, batch, _ = _mods()
    worlds = _worlds()
    steps = [30, 44, 18, 60, 26]
    eng = batch.BatchEngine(max_worlds=8, pool_bytes=256 << 20)
    slots = [eng.admit(w, sim.Params(nx=w.nx, ny=w.ny), s) for w, s in zip(worlds, steps)]
    while any(eng.remaining(s) > 0 for s in slots):
        eng.advance(10)
    for w, s, st in zip(worlds, slots, steps):
        got = eng.retire(s, w)
        assert _same(got, _alone(sim, w, st)), (w.nx, w.ny, st)
        _check_oracle(sim, w, got, st, f"batch {w.nx}x{w.ny} N={w.n_particles}")


def test_batch_pool_exhaustion_and_slot_limit():
    sim, batch, _ = _mods()
    w = wl.random_world(3, 128, 128, [30] * 10, amp=0.5)
    p = sim.Params(nx=w.nx, ny=w.ny)
    need = batch.BatchEngine.world_bytes(p, w.n_filaments, w.n_particles)
    eng = batch.BatchEngine(max_worlds=2, pool_bytes=need * 2 + (8 << 20))
    a = eng.admit(w, p, 10)
    b = eng.admit(w, p, 10)
    with pytest.raises(sim.SimError) as ei:
        eng.admit(w, p, 10)
    assert ei.value.status in (sim.SIM_E_FULL, sim.SIM_E_WORKSPACE)
    eng.advance(10)
    eng.retire(a, w)
    c = eng.admit(w, p, 4)                  # the freed slot and memory are reused
    eng.advance(4)
    eng.retire(b, w)
    eng.retire(c, w)


def test_unstable_world_flagged_alone():
    sim, batch, _ = _mods()
    good = wl.random_world(1, 64, 64, [20], amp=0.5)
    bad = wl.random_world(2, 64, 64, [20], amp=0.5)
    eng = batch.BatchEngine(max_worlds=4, pool_bytes=64 << 20)
    sg = eng.admit(good, sim.Params(nx=64, ny=64), 20)
    sb = eng.admit(bad, sim.Params(nx=64, ny=64, u_max=1e-9), 20)
    eng.advance(20)
    with pytest.raises(sim.SimError) as ei:
        eng.retire(sb, bad)
    assert ei.value.status == sim.SIM_E_UNSTABLE
    assert _same(eng.retire(sg, good), _alone(sim, good, 20))


def test_served_results_equal_alone_runs():
    sim, batch, serve = _mods()
    jobs = wl.served_jobs(0, n_jobs=10, rate=200.0, max_fil=40, len_range=(8, 48), side_range=(64, 128),
                          steps_range=(20, 80))
    pf = lambda job: sim.Params(nx=job.world.nx, ny=job.world.ny)
    need = [batch.BatchEngine.world_bytes(pf(j), j.world.n_filaments, j.world.n_particles) for j in jobs]
    # a budget that holds about three jobs at a time forces queueing
    eng = batch.BatchEngine(max_worlds=4, pool_bytes=int(3.2 * max(need)) + (8 << 20))
    srv = serve.Server(serve.GpuExecutor(eng, pf), chunk_steps=10)
    stats = srv.run(jobs)
    assert all(r.ok for r in stats.results), [r.error for r in stats.results]
    assert stats.peak_resident >= 2
    for job, r in zip(jobs, stats.results):
        assert _same(r.state, _alone(sim, job.world, job.steps)), job.job_id
        _check_oracle(sim, job.world, r.state, job.steps, f"served job {job.job_id}")
    print("served:", stats.summary())


def test_live_submissions_match_oracle():
    """Jobs submitted by a producer thread while the loop runs: every result
    equals the same world run alone (bitwise) and matches the oracle."""
    import threading
    sim, batch, serve = _mods()
    jobs = wl.served_jobs(1, n_jobs=8, rate=200.0, max_fil=30, len_range=(8, 40), side_range=(64, 96),
                          steps_range=(20, 60))
    pf = lambda job: sim.Params(nx=job.world.nx, ny=job.world.ny)
    need = max(batch.BatchEngine.world_bytes(pf(j), j.world.n_filaments, j.world.n_particles) for j in jobs)
    eng = batch.BatchEngine(max_worlds=4, pool_bytes=int(3.2 * need) + (8 << 20))
    srv = serve.Server(serve.GpuExecutor(eng, pf), chunk_steps=10)
    futs = []

    def producer():
        t0 = time.perf_counter()
        for j in jobs:                           # the trace's gaps, in real time
            time.sleep(max(0.0, j.arrival - (time.perf_counter() - t0)))
            futs.append((j, srv.submit(j)))
        srv.close()

    th = threading.Thread(target=producer)
    th.start()
    stats = srv.serve(idle_poll=0.002)
    th.join()
    assert len(futs) == len(jobs) and all(f.result().ok for _, f in futs)
    for job, f in futs:
        r = f.result()
        assert _same(r.state, _alone(sim, job.world, job.steps)), job.job_id
        _check_oracle(sim, job.world, r.state, job.steps, f"live job {job.job_id}")
    print("live:", stats.summary())


def test_autotuner_picks_a_measured_setting(tmp_path, monkeypatch):
    sim, batch, _ = _mods()
    from paper_2607_02954_amd import autotune
    monkeypatch.setenv("MICROCOSM_CACHE", str(tmp_path))
    worlds = _worlds()[:3]
    best, table = autotune.tune(worlds, lambda w: sim.Params(nx=w.nx, ny=w.ny), 256 << 20, steps_per_trial=20,
                                candidates={"chunk_steps": [10, 20], "cell_blocks": [512, 2048],
                                            "node_blocks": [256, 1024]})
    assert len(table) == 8 and best in table
    assert best["ms_per_step"] == min(r["ms_per_step"] for r in table)
    again, t2 = autotune.tune(worlds, lambda w: sim.Params(nx=w.nx, ny=w.ny), 256 << 20)
    assert again == best and t2 == []       # served from the cache


def test_tile_tuner_picks_measured_side_per_class():
    sim, batch, _ = _mods()
    from paper_2607_02954_amd import autotune
    worlds = _worlds()
    policy, table = autotune.tune_tiles(worlds, lambda w: sim.Params(nx=w.nx, ny=w.ny), 256 << 20,
                                        steps_per_trial=20)
    classes = {autotune.grid_class(w) for w in worlds}
    per_class = [r for r in table if r["class"] != "all"]
    assert len(per_class) == 3 * len(classes)
    whole = [r for r in table if r["class"] == "all"]
    assert whole and whole[0]["policy"] == "per class"
    print("tile tuning:", table)
    best = min(whole, key=lambda r: r["ms_per_step"])["policy"]
    if best == "per class":
        for cls in classes:
            rows = [r for r in per_class if r["class"] == cls]
            assert policy.sides[cls] == min(rows, key=lambda r: r["ms_per_step"])["tile"]
    else:
        assert policy.sides == {} and policy.default == int(best.split()[1])
    # worlds run with the chosen sides still equal their alone runs
    w = worlds[2]
    p = policy.params(w)
    eng = batch.BatchEngine(max_worlds=2, pool_bytes=64 << 20)
    s = eng.admit(w, p, 20)
    eng.advance(20)
    got = eng.retire(s, w)
    assert _same(got, _alone(sim, w, 20, tile=p.tile))
