"""Benchmark: particle-steps/s of the filament-fluid step on one MI355X.

Workload (default): 1,048,576 nodes in chains of U{16..256} nodes on a
2048 x 2048 periodic grid, active bending (0.5 rad, period U(20, 100) steps),
FP32, seed 0.  A step is one pass of the whole hot path (actuation, PBD
elastic force, deposit, Gaussian filter, repulsion, force spread, D2Q9 TRT
fluid update, gather + integrate).  Inputs are resident in HBM before the
timed region; the timed region is K steps of sim_rollout (captured graphs).

Prints one JSON line.  Also reports the deterministic sorted-segment and the
direct-atomic transfer variants, a live per-kernel timing of the dominant
(fluid) kernel against the HBM roofline, the differentiation workload
(backward / forward cost), the batched + served workload (rollouts/s and
p50/p99 latency against the plain per-world path), and the FP64 oracle on a
bounded sample of host-CPU work.
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import threading
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2607_02954_amd import sim, workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0
# dominant kernel: the fluid update k_lbm, which per launch must move the
# populations (read + write, 72 B/cell), the grid force (read, 8 B/cell) and
# the velocity (write, 8 B/cell)
FLUID_BYTES_PER_CELL = 88
STEP_BYTES_PER_CELL = 120     # whole-step algorithmic bytes per cell
STEP_BYTES_PER_NODE = 24      # whole-step algorithmic bytes per node
KERNELS = ["elastic", "bin_or_sort", "filter", "repulse_spread", "fluid", "integrate"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_lbm_scaling_2048.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2607_02954_amd", "csrc", n)
                  for n in ("kernels.hip", "device_util.h", "engine.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None when the kernel sources changed since the counters were taken."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != kernel_source_hash():
        return None
    return d["bytes_per_launch"]


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


GRAPH_CHUNK = 20              # steps per captured chunk graph of a single world


def time_rollout(W, warmup, steps, t0=0):
    """Seconds for `steps` steps of sim_rollout after `warmup` untimed steps.

    The untimed part runs at least one chunk and one step pair, so every graph
    the timed rollout launches (the chunk graph and the pair graph) has been
    captured and instantiated before the start event: capture is set-up, not
    step work."""
    W.rollout(t0, max(warmup, GRAPH_CHUNK + 2))
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    W.rollout(t0 + max(warmup, GRAPH_CHUNK + 2), steps)
    end.record()
    torch.cuda.synchronize()
    W.sync()
    return start.elapsed_time(end) / 1000.0


def bench_served(seed, pool_gib, tune_steps):
    """Served workload: 256 rollout jobs (filament counts log-uniform 1..512,
    lengths U{8..128}, grids 128^2..512^2, 200..2000 steps), Poisson arrivals
    at 50 jobs/s, continuous batching through one pool of world slots.

    Also runs the same jobs (a) all arrived at once through the same batch
    engine (throughput capacity) and (b) one at a time through the plain
    per-world sim_rollout path, whose FIFO latencies under the same arrivals
    are replayed from the measured per-job times.  Every served result is
    compared bitwise with its per-world run."""
    from dataclasses import replace
    from paper_2607_02954_amd import autotune, batch, serve

    jobs = wl.served_jobs(seed)
    pool_bytes = int(pool_gib * (1 << 30))
    # tuning on a representative scratch batch (every 8th job): the tile side
    # per grid-size class first, then chunk and block counts with those sides
    rep = [j.world for j in jobs[::8]]
    policy, tile_table = autotune.tune_tiles(rep, lambda w: sim.Params(nx=w.nx, ny=w.ny), pool_bytes,
                                             steps_per_trial=tune_steps)
    log(f"served: tile sides per class {policy.sides}, otherwise {policy.default}")
    pf = lambda job: policy.params(job.world)
    best, table = autotune.tune(rep, policy.params, pool_bytes,
                                steps_per_trial=tune_steps, use_cache=False,
                                candidates={"chunk_steps": [10, 20, 40], "cell_blocks": [2048, 4096, 8192],
                                            "node_blocks": [1024, 2048]})
    torch.cuda.empty_cache()

    def run(js, live=False):
        eng = batch.BatchEngine(max_worlds=len(js), pool_bytes=pool_bytes)
        eng.set_tuning(best["chunk_steps"], best["cell_blocks"], best["node_blocks"])
        srv = serve.Server(serve.GpuExecutor(eng, pf), chunk_steps=best["chunk_steps"])
        torch.cuda.synchronize()
        if live:
            # a producer thread submits each job at its Poisson arrival time
            # while the loop runs on this thread
            def producer():
                t0 = time.perf_counter()
                for j in sorted(js, key=lambda j: j.arrival):
                    time.sleep(max(0.0, j.arrival - (time.perf_counter() - t0)))
                    srv.submit(j)
                srv.close()
            th = threading.Thread(target=producer)
            th.start()
            stats = srv.serve(idle_poll=0.001)
            th.join()
            by_id = {r.job_id: r for r in stats.results}
            stats.results = [by_id[j.job_id] for j in js]
        else:
            stats = srv.run(js)
        torch.cuda.synchronize()
        eng.close()
        return stats

    log(f"served: tuned {best}")
    served = run(jobs, live=True)
    log(f"served: Poisson run done {served.summary()['makespan_s']:.2f} s")
    offline = run([replace(j, arrival=0.0) for j in jobs])
    s_sum, o_sum = served.summary(), offline.summary()
    log("served: all-arrived run done; per-world runs next")

    # plain per-world path, one job at a time
    service, equal = [], 0
    for job, r in zip(jobs, served.results):
        t0 = time.perf_counter()
        W = sim.World(job.world, pf(job))
        W.rollout(0, job.steps)
        W.sync()
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        if r.ok and all(torch.equal(getattr(W.state, k), getattr(r.state, k)) for k in ("cell", "frac", "f", "u")):
            equal += 1
        W.close()
        del W
        r.state = None
    finish, lat = 0.0, []
    for job, s in zip(sorted(jobs, key=lambda j: j.arrival), [service[j.job_id] for j in
                                                               sorted(jobs, key=lambda j: j.arrival)]):
        finish = max(finish, job.arrival) + s
        lat.append(finish - job.arrival)
    total = float(sum(service))
    steps = sum(j.steps for j in jobs)
    return {
        "workload": "256 served rollout jobs: filaments log-uniform 1..512, lengths U{8..128}, "
                    "grids 128^2..512^2 (step 32), 200..2000 steps, Poisson arrivals 50 jobs/s",
        "submission": "live: a producer thread submits each job at its arrival time while the loop runs",
        "world_steps": steps,
        "particle_steps": int(sum(j.world.n_particles * j.steps for j in jobs)),
        "pool_bytes": pool_bytes,
        "tuning": best,
        "tile_side_per_grid_class": policy.sides,
        "tile_side_default": policy.default,
        "tile_tuning": tile_table,
        "served": {k: s_sum[k] for k in ("completed", "rollouts_per_s", "p50_latency_s", "p99_latency_s",
                                         "makespan_s", "chunks", "peak_resident", "peak_bytes")},
        "batched_all_arrived": {k: o_sum[k] for k in ("completed", "rollouts_per_s", "p50_latency_s",
                                                      "p99_latency_s", "makespan_s", "chunks")},
        "per_world": {
            "rollouts_per_s": len(jobs) / total,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "busy_s": total,
            "latency": "FIFO replay of the measured per-job times under the same arrivals",
        },
        "batched_vs_per_world_throughput": o_sum["rollouts_per_s"] * total / len(jobs),
        "served_equal_to_per_world_bitwise": f"{equal}/{len(jobs)}",
    }


def _differentiation_times(w, p, n, k, reps):
    """Median plain rollout, checkpointed forward and backward times (ms) of
    one world over n steps (checkpoints every k), and the last loss."""
    W = sim.World(w, p)
    tgt = torch.tensor(w.target, dtype=torch.float64, device="cuda")
    cell0, frac0 = W.state.cell.clone(), W.state.frac.clone()

    def reset():
        W.state.cell.copy_(cell0)
        W.state.frac.copy_(frac0)
        W.state.f.zero_()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    plain, fwd, bwd = [], [], []
    for r in range(reps + 1):
        reset()
        torch.cuda.synchronize()
        ev[0].record()
        W.rollout(0, n)
        ev[1].record()
        torch.cuda.synchronize()
        reset()
        ra = torch.tensor(w.rest_angle, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        ev[2].record()
        xT = sim.Rollout.apply(ra, W, 0, n, k)
        loss = ((xT - tgt) ** 2).sum() / xT.shape[1]
        ev[3].record()
        torch.cuda.synchronize()
        b0 = torch.cuda.Event(enable_timing=True)
        b1 = torch.cuda.Event(enable_timing=True)
        b0.record()
        loss.backward()
        b1.record()
        torch.cuda.synchronize()
        if r:                                    # first repetition warms up
            plain.append(ev[0].elapsed_time(ev[1]))
            fwd.append(ev[2].elapsed_time(ev[3]))
            bwd.append(b0.elapsed_time(b1))
    W.close()
    return float(np.median(plain)), float(np.median(fwd)), float(np.median(bwd)), float(loss.detach())


def bench_adjoint(seed, reps=5):
    """Differentiation workload: 64 chains x 48 nodes on 256^2, 200 steps,
    checkpoints every 20; loss = mean squared distance to the seeded target
    fold; gradient in the rest angles through the autograd Function.  Also
    the same with the coupling's leakage fixes (3 MDF iterations, two marker
    layers 0.5 cells apart, both), and 16 such worlds as one set."""
    from dataclasses import replace as dc_replace
    w = wl.folding_population(seed)
    p = sim.Params(nx=w.nx, ny=w.ny)
    n, k = 200, 20
    pm, fm, bm, loss = _differentiation_times(w, p, n, k, reps)
    out = {
        "workload": "folding: 64 chains x 48 nodes on 256x256, 200 steps, checkpoints every 20, "
                    "gradient of the target-fold loss in the rest angles",
        "plain_rollout_ms": pm,
        "checkpointed_forward_ms": fm,
        "backward_ms": bm,
        "bwd_over_fwd": bm / fm,
        "bwd_over_plain_fwd": bm / pm,
        "loss": loss,
    }
    variants = {}
    for name, kw in (("mdf3", dict(mdf_iters=3)), ("two_layer", dict(marker_offset=0.5)),
                     ("mdf3_two_layer", dict(mdf_iters=3, marker_offset=0.5))):
        vp, vf, vb, vl = _differentiation_times(w, dc_replace(p, **kw), n, k, max(2, reps // 2))
        variants[name] = {"checkpointed_forward_ms": vf, "backward_ms": vb, "bwd_over_fwd": vb / vf, "loss": vl}
        log(f"differentiation {name}: forward {vf:.2f} ms, backward {vb:.2f} ms")
    out["coupling_variants"] = variants
    out["set_of_worlds"] = bench_adjoint_set(seed, n, k, fm + bm, reps=max(2, reps // 2))
    return out


def bench_adjoint_scale(world, tile, n=20, k=10, reps=3):
    """Reverse mode at the full workload (1,048,576 nodes on 2048^2): one
    checkpointed rollout of n steps (checkpoints every k) and its backward,
    loss = mean squared distance of the final positions to a seeded target."""
    W = sim.World(world, sim.Params(nx=world.nx, ny=world.ny, tile=tile))
    x0 = world.positions64()
    tgt = torch.tensor(x0 + np.random.default_rng(7).normal(0, 0.5, size=x0.shape), dtype=torch.float64,
                       device="cuda")
    cell0, frac0 = W.state.cell.clone(), W.state.frac.clone()
    fwd, bwd = [], []
    for r in range(reps + 1):
        W.state.cell.copy_(cell0)
        W.state.frac.copy_(frac0)
        W.state.f.zero_()
        ra = torch.tensor(world.rest_angle, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        xT = sim.Rollout.apply(ra, W, 0, n, k)
        loss = ((xT - tgt) ** 2).sum() / xT.shape[1]
        e[1].record()
        loss.backward()
        e[2].record()
        torch.cuda.synchronize()
        if r:
            fwd.append(e[0].elapsed_time(e[1]))
            bwd.append(e[1].elapsed_time(e[2]))
    W.close()
    fm, bm = float(np.median(fwd)), float(np.median(bwd))
    return {"workload": f"scaling: {world.n_particles} nodes on {world.nx}x{world.ny}, {n} steps, checkpoints every "
                        f"{k}, gradient of a target-position loss in the rest angles",
            "checkpointed_forward_ms": fm, "backward_ms": bm, "bwd_over_fwd": bm / fm,
            "backward_ms_per_step": bm / n}


def bench_adjoint_set(seed, n, k, alone_ms, n_worlds=16, reps=2):
    """The same differentiation for 16 folding worlds (seeds seed..seed+15)
    stepped and reversed together as one set of worlds (sim_create_set): one
    forward with checkpoints and one backward for all of them, against 16
    times the single world's forward + backward."""
    worlds = [wl.folding_population(seed + i) for i in range(n_worlds)]
    p = sim.Params(nx=worlds[0].nx, ny=worlds[0].ny)
    S = sim.WorldSet(worlds, p)
    tg = [torch.tensor(w.target, dtype=torch.float64, device="cuda") for w in worlds]
    init = [(st.cell.clone(), st.frac.clone()) for st in S.states]
    ra0 = torch.tensor(np.concatenate([w.rest_angle for w in worlds]), dtype=torch.float64, device="cuda")
    times = []
    for r in range(reps + 1):
        for st, (c0, f0) in zip(S.states, init):
            st.cell.copy_(c0)
            st.frac.copy_(f0)
            st.f.zero_()
        ra = ra0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = sim.SetRollout.apply(ra, S, 0, n, k)
        off, loss = 0, 0.0
        for t, m in zip(tg, S.n_parts):
            loss = loss + ((x[off:off + 2 * m].reshape(2, m) - t) ** 2).sum() / m
            off += 2 * m
        loss.backward()
        torch.cuda.synchronize()
        if r:
            times.append(1000.0 * (time.perf_counter() - t0))
    S.close()
    ms = float(np.median(times))
    return {"worlds": n_worlds, "forward_plus_backward_ms": ms, "per_world_ms": ms / n_worlds,
            "alone_per_world_ms": alone_ms, "speedup_over_alone": alone_ms * n_worlds / ms}


def bench_density_folding(seed, reps=3):
    """The paper's folding objective at its sizes: one 1000-node filament on
    256^2, 250 steps with checkpoints every 25, loss = mean squared error of
    the Gaussian-splatted density (128 x 128 image, sigma 2 cells) to a seeded
    target image; gradient in the rest angles (autograd: DensityLoss after
    Rollout)."""
    w = wl.density_folding(seed)
    n, k, sigma, amp = 250, 25, 2.0, 0.1
    W = sim.World(w, sim.Params(nx=w.nx, ny=w.ny))
    T = torch.tensor(w.meta["image"], dtype=torch.float32, device="cuda")
    cell0, frac0 = W.state.cell.clone(), W.state.frac.clone()
    fwd, bwd = [], []
    for r in range(reps + 1):
        W.state.cell.copy_(cell0)
        W.state.frac.copy_(frac0)
        W.state.f.zero_()
        ra = torch.tensor(w.rest_angle, dtype=torch.float64, device="cuda", requires_grad=True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        ev[0].record()
        xT = sim.Rollout.apply(ra, W, 0, n, k)
        loss = sim.DensityLoss.apply(xT, w.nx, w.ny, T, sigma, amp)
        ev[1].record()
        loss.backward()
        ev[2].record()
        torch.cuda.synchronize()
        if r:
            fwd.append(ev[0].elapsed_time(ev[1]))
            bwd.append(ev[1].elapsed_time(ev[2]))
    W.close()
    fm, bm = float(np.median(fwd)), float(np.median(bwd))
    return {
        "workload": "density folding: one 1000-node filament on 256x256, 250 steps, checkpoints every 25, "
                    "loss = MSE of the Gaussian-splatted density (128x128 image, sigma 2 cells) to a seeded "
                    "target image, gradient in the rest angles",
        "forward_ms": fm, "backward_ms": bm, "bwd_over_fwd": bm / fm, "loss": float(loss.detach()),
        "grad_norm": float(ra.grad.norm()),
    }


def host_cpu():
    """Host CPU model and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def oracle_rate(world, steps, threads):
    """Particle-steps/s of the FP64 oracle (unchanged) on `threads` host
    threads over `steps` steps, after one untimed step (first touch)."""
    import oracle as O
    prev = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        p = O.Params(nx=world.nx, ny=world.ny)
        inp = O.inputs_from_world(world)
        x = O.positions_from_world(world)
        f = O.rest_populations(p)
        with torch.no_grad():
            x, f, _ = O.step(x, f, 0, inp, p)
            t0 = time.perf_counter()
            for k in range(steps):
                x, f, _ = O.step(x, f, 1 + k, inp, p)
            dt = time.perf_counter() - t0
    finally:
        torch.set_num_threads(prev)
    return world.n_particles * steps / dt, dt


def cpu_baseline(world, sample_steps, single_steps):
    """The FP64 oracle on the host cores for a bounded number of steps, with
    every usable core and with one."""
    model, nproc, usable = host_cpu()
    v_all, dt_all = oracle_rate(world, sample_steps, usable)
    v_one, dt_one = oracle_rate(world, single_steps, 1) if single_steps > 0 else (None, 0.0)
    return {
        "value": v_all,
        "unit": "particle-steps/s",
        "cores": usable,
        "kind": "oracle",
        "sample": f"{sample_steps} steps of the same workload after one untimed step "
                  f"({dt_all:.1f} s, float64, torch CPU, {usable} threads)",
        "single_thread": {"value": v_one, "steps": single_steps, "seconds": dt_one},
        "host": {"cpu_model": model, "nproc": nproc, "usable_cores": usable},
    }


def bench_widened(world, seed, tile, steps, warmup):
    """The coupling, field and topology extensions timed against the plain
    step on the same worlds (ms/step over `steps` captured steps each):

    * MDF and two-layer markers: a quarter of the million-node workload's
      nodes (262,144: lengths U{16..256}) on the same 2048^2 grid, with
      explicit coupling and with 4 MDF iterations, each on one layer and on
      two markers offset 0.5 cells along the normal, on the binned and on
      the direct transfer; 100 steps each (at the full workload's density
      the MDF iteration diverges where markers crowd, a limit of the
      method);
    * energy field (binned transfer): the same workload with a field of 4096
      Gaussian packets (amplitudes U(0.5, 2), widths U(3, 12) cells) that the
      nodes deplete at rate 0.05 per step;
    * topology generality (binned): the workload with per-edge stiffness
      arrays U(0.2, 1), a world of chains plus closed loops (lengths
      U{16..64}, 10% of the nodes) of the same size with stiffness arrays,
      and about a million nodes of branched creatures;
      plus one rest-effort reduction (the descriptors of a rest-value change)
      over the million nodes."""
    from dataclasses import replace as dc_replace
    N = world.n_particles
    base = sim.Params(nx=world.nx, ny=world.ny, tile=tile)
    out = {}

    def timed(w, p, n, label):
        W = sim.World(w, p)
        secs = time_rollout(W, warmup, n)
        W.close()
        del W
        torch.cuda.empty_cache()
        ms = 1000.0 * secs / n
        log(f"widened {label}: {ms:.4f} ms/step")
        return {"ms_per_step": ms, "value": w.n_particles * n / secs}

    # MDF and two-layer markers, direct transfer
    wq = wl.random_world(seed, world.nx, world.ny, wl.scaling_lengths(seed, N // 4), amp=0.5)
    direct = dc_replace(base, transfer="direct")
    rows = {"binned_explicit": timed(wq, base, 100, "quarter binned explicit"),
            "binned_mdf4": timed(wq, dc_replace(base, mdf_iters=4), 100, "quarter binned mdf4"),
            "binned_two_layer": timed(wq, dc_replace(base, marker_offset=0.5), 100, "quarter binned two layers"),
            "binned_mdf4_two_layer": timed(wq, dc_replace(base, mdf_iters=4, marker_offset=0.5), 100,
                                           "quarter binned mdf4 two layers"),
            "explicit": timed(wq, direct, 100, "quarter direct explicit"),
            "mdf4": timed(wq, dc_replace(direct, mdf_iters=4), 100, "quarter direct mdf4"),
            "mdf4_two_layer": timed(wq, dc_replace(direct, mdf_iters=4, marker_offset=0.5), 100,
                                    "quarter direct mdf4 two layers")}
    for k in ("mdf4", "mdf4_two_layer"):
        rows[k]["over_explicit"] = rows[k]["ms_per_step"] / rows["explicit"]["ms_per_step"]
    for k in ("binned_mdf4", "binned_two_layer", "binned_mdf4_two_layer"):
        rows[k]["over_explicit"] = rows[k]["ms_per_step"] / rows["binned_explicit"]["ms_per_step"]
    out["coupling"] = dict(workload=f"{wq.n_particles} nodes (lengths U{{16..256}}) on {wq.nx}x{wq.ny}, "
                                    "100 steps", **rows)

    # energy field, binned transfer
    g = np.random.default_rng(seed + 104729)
    P = 4096
    c = torch.tensor(g.uniform(0.0, 1.0, size=(2, P)) * np.array([[world.nx], [world.ny]]), dtype=torch.float32,
                     device="cuda")
    a = torch.tensor(g.uniform(0.5, 2.0, size=P), dtype=torch.float32, device="cuda")
    wd = torch.tensor(g.uniform(3.0, 12.0, size=P), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E = sim.energy_packets(world.nx, world.ny, c, a, wd)
    torch.cuda.synchronize()
    packets_ms = 1000.0 * (time.perf_counter() - t0)
    plain = timed(world, base, steps, "binned plain")
    we = copy.copy(world)
    we.energy = E.cpu().numpy()
    del E
    field = timed(we, dc_replace(base, energy_rate=0.05), steps, "binned energy")
    out["energy"] = {"workload": f"scaling workload, binned, {P} packets, rate 0.05", "plain": plain, "field": field,
                     "over_plain": field["ms_per_step"] / plain["ms_per_step"], "packets_build_ms": packets_ms}

    # topology generality, binned transfer
    ws = copy.copy(world)
    ws.stiffness = tuple(g.uniform(0.2, 1.0, size=N).astype(np.float32) for _ in range(3))
    stiff = timed(ws, base, steps, "binned per-edge stiffness")
    n_loop = N // 10
    loops = []
    while n_loop - sum(loops) >= 64 + 16:
        loops.append(int(g.integers(16, 65)))
    loops.append(n_loop - sum(loops))            # 16..79 nodes
    wg = wl.generality_world(seed, world.nx, world.ny, wl.scaling_lengths(seed, N - sum(loops)), loops)
    gen = timed(wg, base, steps, "binned loops + stiffness")
    del wg
    wb = wl.branched_world(seed, world.nx, world.ny, 26500)
    branched = timed(wb, base, steps, "binned branched creatures")
    branched["nodes"] = wb.n_particles
    branched["filaments"] = wb.n_filaments
    branched["attachments"] = int((wb.parent >= 0).sum())
    del wb
    dev = sim.DeviceState(ws, "cuda")
    ra2 = dev.rest_angle + 0.01
    rl2 = dev.rest_length * 1.01
    sim.rest_effort(dev, ra2, rl2)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(10):
        sim.rest_effort(dev, ra2, rl2)
    ev[1].record()
    torch.cuda.synchronize()
    eff_ms = ev[0].elapsed_time(ev[1]) / 10
    del dev
    torch.cuda.empty_cache()
    out["topology"] = {"workload": "scaling workload; loops world: same node count, 10% of the nodes in loops "
                                   f"({len(loops)} loops of U{{16..64}} nodes); branched world: 26,500 creatures "
                                   "(a chain or loop with chains hanging from its nodes) on the same grid",
                       "plain": plain, "per_edge_stiffness": stiff, "loops_and_stiffness": gen,
                       "branched_creatures": branched,
                       "stiffness_over_plain": stiff["ms_per_step"] / plain["ms_per_step"],
                       "loops_over_plain": gen["ms_per_step"] / plain["ms_per_step"],
                       "branched_over_plain": branched["ms_per_step"] / plain["ms_per_step"],
                       "rest_effort_ms": eff_ms}
    return out


def bench_small_configs(seed, steps_c1, steps_c2, cpu_c1, cpu_c2, with_cpu):
    """The parity configuration (one 32-node chain on 64^2) and the uniform
    population (1024 chains x 64 nodes on 512^2, active bending): particle-
    steps/s of the captured-graph rollout, the oracle beside each."""
    out = {}
    model, nproc, usable = host_cpu()
    for name, world, steps, cpu_steps in (
            ("parity_32_nodes_64x64", wl.parity_single(seed), steps_c1, cpu_c1),
            ("uniform_65536_nodes_512x512", wl.uniform_population(seed), steps_c2, cpu_c2)):
        W = sim.World(world, sim.Params(nx=world.nx, ny=world.ny))
        secs = time_rollout(W, GRAPH_CHUNK, steps)
        W.close()
        del W
        N = world.n_particles
        rec = {"particles": N, "grid": [world.nx, world.ny], "steps": steps,
               "ms_per_step": 1000.0 * secs / steps, "value": N * steps / secs,
               "unit": "particle-steps/s",
               "step_GBs": (STEP_BYTES_PER_CELL * world.nx * world.ny + STEP_BYTES_PER_NODE * N)
                           / (secs / steps) / 1e9}
        if with_cpu:
            v_all, dt_all = oracle_rate(world, cpu_steps, usable)
            v_one, dt_one = oracle_rate(world, max(1, cpu_steps // 4), 1)
            rec["oracle"] = {"value": v_all, "cores": usable, "steps": cpu_steps, "seconds": dt_all,
                             "single_thread_value": v_one, "single_thread_steps": max(1, cpu_steps // 4)}
        out[name] = rec
        log(f"{name}: {rec['ms_per_step']:.4f} ms/step")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--cpu-single-steps", type=int, default=1)
    ap.add_argument("--no-small", action="store_true", help="skip the 64^2 and 512^2 configurations")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sorted", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-widened", action="store_true",
                    help="skip the coupling, energy-field and topology extensions")
    ap.add_argument("--pool-gib", type=float, default=8.0, help="HBM budget of the served pool")
    ap.add_argument("--tune-steps", type=int, default=20)
    ap.add_argument("--tile", type=int, default=0, choices=[0, 16, 32, 64],
                    help="grid tile side of the scaling workload (0: the autotuner's choice)")
    ap.add_argument("--probe-atomics", action="store_true",
                    help="only measure the atomic-add throughput of the device (sim_measure_atomics)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: a world or a batch of worlds runs on one device; "
                                   "--gpus must be 1"}))
        sys.exit(2)
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)

    if args.probe_atomics:
        print(json.dumps(sim.measure_atomics()), flush=True)
        return

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        # the same copy timed (read + write bytes over the launch time): the
        # HBM rate a plain streaming kernel reaches on this device
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        t0.record()
        for _ in range(reps):
            b.copy_(a)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        print(json.dumps({"calibration_copy_bytes_each_way": n * 4, "launches": 3 + reps,
                          "copy_ms": ms, "copy_GBs": 2 * n * 4 / (ms * 1e-3) / 1e9}), flush=True)
        return

    world = wl.scaling_population(args.seed)
    N, ncell = world.n_particles, world.nx * world.ny
    # the autotuner's tile side for this world (each side timed over 40 steps)
    if args.tile:
        tile, tile_rows = args.tile, []
    else:
        from paper_2607_02954_amd import autotune
        tile, tile_rows = autotune.tune_world_tile(world, sim.Params(nx=world.nx, ny=world.ny), steps=40)
        torch.cuda.empty_cache()
    log(f"scaling workload: tile side {tile} {tile_rows}")
    W = sim.World(world, sim.Params(nx=world.nx, ny=world.ny, tile=tile))
    secs = time_rollout(W, args.warmup, args.steps)
    ms_step = 1000.0 * secs / args.steps
    value = N * args.steps / secs
    # live per-kernel timing on the world's stream, same state; the fluid
    # kernel's time comes from its dispatch's own start and end timestamps
    t_next = max(args.warmup, GRAPH_CHUNK + 2) + args.steps
    kms = W.profile(t_next, args.profile_steps)
    fluid_ms = kms[4]
    fluid_bytes = FLUID_BYTES_PER_CELL * ncell
    fluid_gbs = fluid_bytes / (fluid_ms * 1e-3) / 1e9
    step_bytes = STEP_BYTES_PER_CELL * ncell + STEP_BYTES_PER_NODE * N
    W.close()
    del W
    torch.cuda.empty_cache()

    variants = {}
    if not args.no_sorted:
        for mode in ("sorted", "direct"):
            Ws = sim.World(world, sim.Params(nx=world.nx, ny=world.ny, transfer=mode, tile=tile))
            s_secs = time_rollout(Ws, args.warmup, args.steps)
            skms = Ws.profile(t_next, args.profile_steps)
            variants[mode] = {
                "value": N * args.steps / s_secs,
                "ms_per_step": 1000.0 * s_secs / args.steps,
                "kernel_ms": dict(zip(KERNELS, [round(v, 5) for v in skms])),
            }
            Ws.close()
            del Ws

    out = {
        "metric": "particle-steps/s (1M particles)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "graph_warmup_steps": max(args.warmup, GRAPH_CHUNK + 2),
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded chains, uniform centres and orientations)",
        "config": {
            "workload": "scaling: 1,048,576 nodes, chain lengths U{16..256}, 2048x2048 periodic grid, "
                        "active bending 0.5 rad, tile-binned particle-to-grid transfer",
            "particles": N, "filaments": world.n_filaments, "grid": [world.nx, world.ny],
            "seed": args.seed, "tile_side": tile,
        },
        "tile_tuning": tile_rows,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_lbm (D2Q9 TRT fluid update with Guo forcing)",
            "achieved": fluid_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": fluid_gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "kernel_ms": fluid_ms,
            "bytes_per_launch": fluid_bytes,
        },
        "step_roofline": {
            "algorithmic_bytes_per_step": step_bytes,
            "achieved_GBs": step_bytes / (ms_step * 1e-3) / 1e9,
            "frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "kernel_ms": dict(zip(KERNELS, [round(v, 5) for v in kms])),
        "transfer_variants": variants,
    }
    log(f"scaling workload done: {ms_step:.4f} ms/step")
    # the atomic adds the transfers are built on: LDS float vs integer adds
    # (the binned transfer sums in 64-bit fixed point) and global float
    # atomics (the direct transfer), with the direct transfer's own rate
    at = sim.measure_atomics()
    if "direct" in variants:
        kd = variants["direct"]["kernel_ms"]
        # direct mode: 16 deposit atomics per node in the elastic kernel and
        # 32 spread atomics per node in the repulsion kernel
        at["direct_transfer_atomics_per_s"] = 48 * N / ((kd["elastic"] + kd["repulse_spread"]) * 1e-3)
    out["atomic_throughput"] = at
    if not args.no_adjoint:
        out["differentiation"] = bench_adjoint(args.seed)
        out["differentiation"]["at_scale"] = bench_adjoint_scale(world, tile)
        log("differentiation done")
        out["density_folding"] = bench_density_folding(args.seed)
        log("density folding done")
    if not args.no_widened:
        out["widened"] = bench_widened(world, args.seed, tile, args.steps, args.warmup)
        log("widened rows done")
    if not args.no_served:
        out["batched_served"] = bench_served(args.seed, args.pool_gib, args.tune_steps)
        log("served done")
    if not args.no_small:
        out["small_configs"] = bench_small_configs(args.seed, 1000, 1000, 200, 8, not args.no_cpu)
        log("small configurations done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(world, args.cpu_steps, args.cpu_single_steps)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
