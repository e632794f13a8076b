"""Autotuner for the batched launch: chooses the steps per captured chunk and
the persistent grid sizes of the tile/cell kernels and the node kernels by
timing candidate settings on a scratch batch of representative worlds.

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


def _cache_path() -> str:
    base = os.environ.get("MICROCOSM_CACHE") or os.path.join(
        os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "microcosm")
    return os.path.join(base, "autotune.json")


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
    key = f"{torch.cuda.get_device_name(0)}|{size_class(worlds)}"
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
