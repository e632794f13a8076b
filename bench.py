"""Benchmark: particle-steps/s of the filament-fluid step on one MI355X.

Workload (default): 1,048,576 nodes in chains of U{16..256} nodes on a
2048 x 2048 periodic grid, active bending (0.5 rad, period U(20, 100) steps),
FP32, seed 0.  A step is one pass of the whole hot path (actuation, PBD
elastic force, deposit, Gaussian filter, repulsion, force spread, D2Q9 TRT
fluid update, gather + integrate).  Inputs are resident in HBM before the
timed region; the timed region is K steps of sim_rollout (captured graphs).

Prints one JSON line.  Also reports the deterministic sorted-segment transfer
variant, a live per-kernel timing of the dominant (fluid) kernel against the
HBM roofline, and the FP64 oracle on a bounded sample of host-CPU work.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2607_02954_amd import sim, workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0
FLUID_BYTES_PER_CELL = 88     # populations read + write (72), force read (8), velocity write (8)
STEP_BYTES_PER_CELL = 120     # whole-step algorithmic bytes per cell
STEP_BYTES_PER_NODE = 24      # whole-step algorithmic bytes per node
KERNELS = ["elastic", "bin_or_sort", "filter", "repulse", "fluid", "integrate"]


def time_rollout(W, warmup, steps, t0=0):
    W.rollout(t0, warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    W.rollout(t0 + warmup, steps)
    end.record()
    torch.cuda.synchronize()
    W.sync()
    return start.elapsed_time(end) / 1000.0


def cpu_baseline(world, sample_steps):
    """The FP64 oracle (unchanged) on the host cores for a bounded number of steps."""
    import oracle as O
    p = O.Params(nx=world.nx, ny=world.ny)
    inp = O.inputs_from_world(world)
    x = O.positions_from_world(world)
    f = O.rest_populations(p)
    with torch.no_grad():
        x, f, _ = O.step(x, f, 0, inp, p)        # first-touch warm-up, untimed
        t0 = time.perf_counter()
        for k in range(sample_steps):
            x, f, _ = O.step(x, f, 1 + k, inp, p)
        dt = time.perf_counter() - t0
    return {
        "value": world.n_particles * sample_steps / dt,
        "unit": "particle-steps/s",
        "cores": torch.get_num_threads(),
        "kind": "oracle",
        "sample": f"{sample_steps} steps of the same workload after one untimed step "
                  f"({dt:.1f} s, float64, torch CPU)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sorted", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_each_way": n * 4, "launches": 3}), flush=True)
        return

    world = wl.scaling_population(args.seed)
    N, ncell = world.n_particles, world.nx * world.ny
    W = sim.World(world, sim.Params(nx=world.nx, ny=world.ny))
    secs = time_rollout(W, args.warmup, args.steps)
    ms_step = 1000.0 * secs / args.steps
    value = N * args.steps / secs
    # live per-kernel timing (HIP events on the world's stream), same state
    kms = W.profile(args.warmup + args.steps, args.profile_steps)
    fluid_ms = kms[4]
    fluid_gbs = FLUID_BYTES_PER_CELL * ncell / (fluid_ms * 1e-3) / 1e9
    step_bytes = STEP_BYTES_PER_CELL * ncell + STEP_BYTES_PER_NODE * N
    W.close()
    del W
    torch.cuda.empty_cache()

    variants = {}
    if not args.no_sorted:
        for mode in ("sorted", "direct"):
            Ws = sim.World(world, sim.Params(nx=world.nx, ny=world.ny, transfer=mode))
            s_secs = time_rollout(Ws, args.warmup, args.steps)
            skms = Ws.profile(args.warmup + args.steps, args.profile_steps)
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
            "seed": args.seed,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_lbm (D2Q9 TRT fluid update)",
            "achieved": fluid_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": fluid_gbs / HBM_PEAK_GBS,
            "traffic": None,
            "kernel_ms": fluid_ms,
            "bytes_per_launch": FLUID_BYTES_PER_CELL * ncell,
        },
        "step_roofline": {
            "algorithmic_bytes_per_step": step_bytes,
            "achieved_GBs": step_bytes / (ms_step * 1e-3) / 1e9,
            "frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "kernel_ms": dict(zip(KERNELS, [round(v, 5) for v in kms])),
        "transfer_variants": variants,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(world, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
