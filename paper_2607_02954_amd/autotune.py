"""Autotuner: chooses the grid tile side (16, 32 or 64 cells: the tile of the
filter, spread and integrate kernels and of the node bins) per grid-size
class, then the steps per captured chunk and the persistent grid sizes of
the tile/cell kernels and the node kernels of the batched launch, by timing
candidate settings on scratch worlds.  A single large world gets its tile side
the same way (tune_world_tile).

Results are cached per (device name, size class) in a JSON file so serving
starts with the tuned setting.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, List, Optional, Tuple

import torch

from . import sim
from .batch import BatchEngine

DEFAULT_CANDIDATES = {
    "chunk_steps": [10, 20, 40],
    "cell_blocks": [1024, 2048, 4096, 8192],
    "node_blocks": [512, 1024, 2048, 4096],
}
TILE_SIDES = [16, 32, 64]


def _cache_path() -> str:
    base = os.environ.get("MICROCOSM_CACHE") or os.path.join(
        os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "microcosm")
    return os.path.join(base, "autotune.json")


def grid_class(world) -> str:
    """Size class of one world for the tile choice: log2 of its cell count."""
    return f"cells2^{int(math.log2(max(world.nx * world.ny, 1)))}"


class TilePolicy:
    """Tile side per grid-size class (32 where no class was measured)."""

    def __init__(self, sides: Optional[Dict[str, int]] = None, default: int = 32):
        self.sides = dict(sides or {})
        self.default = default

    def side_for(self, world) -> int:
        return self.sides.get(grid_class(world), self.default)

    def params(self, world, **kw) -> sim.Params:
        return sim.Params(nx=world.nx, ny=world.ny, tile=self.side_for(world), **kw)


def _time_batch(worlds, params_for, pool_bytes, steps, device, chunk=20):
    eng = BatchEngine(max_worlds=len(worlds), pool_bytes=pool_bytes, device=device)
    for w in worlds:
        eng.admit(w, params_for(w), steps=10 ** 9)
    eng.set_tuning(chunk, 4096, 1024)
    eng.advance(chunk)                          # capture + warm
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n = max(chunk, (steps // chunk) * chunk)
    torch.cuda.synchronize()
    start.record()
    eng.advance(n)
    end.record()
    torch.cuda.synchronize()
    eng.close()
    return start.elapsed_time(end) / n


def tune_tiles(worlds: List, params_for, pool_bytes: int, steps_per_trial: int = 40,
               sides: Iterable[int] = TILE_SIDES, device="cuda") -> Tuple[TilePolicy, List[dict]]:
    """Time every tile side on a scratch batch of each grid-size class of
    `worlds` (params_for(w) gives the other parameters; its tile is
    replaced); return the policy (fastest side per class) and the table."""
    from dataclasses import replace
    classes: Dict[str, List] = {}
    for w in worlds:
        classes.setdefault(grid_class(w), []).append(w)
    table, best = [], {}
    for cls, ws in sorted(classes.items()):
        rows = []
        for side in sides:
            ms = _time_batch(ws, lambda w: replace(params_for(w), tile=side), pool_bytes, steps_per_trial, device)
            rows.append({"class": cls, "worlds": len(ws), "tile": side, "ms_per_step": ms})
        table += rows
        best[cls] = min(rows, key=lambda r: r["ms_per_step"])["tile"]
    # every tile side present in a batch is one more launch of each tile
    # kernel per step: the per-class mix is kept only if it beats one side
    # for all worlds on the whole scratch batch
    policies = [("per class", TilePolicy(best))] + [(f"all {s}", TilePolicy({}, default=s)) for s in sides]
    if len(classes) == 1 or len(set(best.values())) == 1:
        policies = policies[:1]
    timed = []
    for name, pol in policies:
        ms = _time_batch(worlds, lambda w: replace(params_for(w), tile=pol.side_for(w)), pool_bytes,
                         steps_per_trial, device)
        table.append({"class": "all", "worlds": len(worlds), "policy": name, "ms_per_step": ms})
        timed.append((ms, pol))
    return min(timed, key=lambda r: r[0])[1], table


def tune_world_tile(world, params: sim.Params, steps: int = 40, sides: Iterable[int] = TILE_SIDES,
                    device="cuda") -> Tuple[int, List[dict]]:
    """Tile side for one (large) world: each side timed over `steps` steps of
    sim_rollout (captured graphs) after one untimed rollout of the same length."""
    from dataclasses import replace
    rows = []
    for side in sides:
        W = sim.World(world, replace(params, tile=side), device=device)
        W.rollout(0, steps)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        W.rollout(steps, steps)
        end.record()
        torch.cuda.synchronize()
        W.sync()
        W.close()
        del W
        rows.append({"tile": side, "ms_per_step": start.elapsed_time(end) / steps})
    return min(rows, key=lambda r: r["ms_per_step"])["tile"], rows


def size_class(worlds) -> str:
    cells = sum(w.nx * w.ny for w in worlds)
    nodes = sum(w.n_particles for w in worlds)
    return f"c2^{int(math.log2(max(cells, 1)))}_n2^{int(math.log2(max(nodes, 1)))}_w{len(worlds)}"


def tune(worlds: List, params_for, pool_bytes: int, steps_per_trial: int = 40,
         candidates: Optional[Dict[str, Iterable[int]]] = None, use_cache: bool = True,
         device="cuda") -> Tuple[dict, List[dict]]:
    """Time every candidate on a scratch batch holding `worlds`; return the
    best setting and the measured table (ms per step)."""
    cand = dict(DEFAULT_CANDIDATES)
    if candidates:
        cand.update({k: list(v) for k, v in candidates.items()})
    tiles = sorted({params_for(w).tile for w in worlds})
    key = f"{torch.cuda.get_device_name(0)}|{size_class(worlds)}|tiles{tiles}"
    path = _cache_path()
    if use_cache and os.path.exists(path):
        try:
            cached = json.load(open(path)).get(key)
            if cached:
                return cached, []
        except (OSError, ValueError):
            pass
    eng = BatchEngine(max_worlds=len(worlds), pool_bytes=pool_bytes, device=device)
    for w in worlds:
        eng.admit(w, params_for(w), steps=10 ** 9)
    table = []
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for chunk in cand["chunk_steps"]:
        n = max(chunk, (steps_per_trial // chunk) * chunk)
        for cb in cand["cell_blocks"]:
            for nb in cand["node_blocks"]:
                eng.set_tuning(chunk, cb, nb)
                eng.advance(chunk)              # capture + warm
                torch.cuda.synchronize()
                start.record()
                eng.advance(n)
                end.record()
                torch.cuda.synchronize()
                table.append({"chunk_steps": chunk, "cell_blocks": cb, "node_blocks": nb,
                              "ms_per_step": start.elapsed_time(end) / n})
    eng.close()
    best = min(table, key=lambda r: r["ms_per_step"])
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            data = json.load(open(path)) if os.path.exists(path) else {}
            data[key] = best
            json.dump(data, open(path, "w"), indent=1)
        except (OSError, ValueError):
            pass
    return best, table
