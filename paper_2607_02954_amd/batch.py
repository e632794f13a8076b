"""Batched worlds on one GPU: many independent worlds of uneven size advanced
by the same kernels in one persistent, graph-captured launch per chunk.

Thin binding over the sim_batch_* entry points.  Device memory for every
resident world comes from one pool tensor, so the pool size is the HBM
budget that admission respects.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import sim
from .sim import SimArrays, check, lib, _ptr


class BatchEngine:
    """A pool of world slots advanced together (sim_batch_*)."""

    def __init__(self, max_worlds: int, pool_bytes: int, device="cuda", stream=None):
        self.device = torch.device(device)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        self.max_worlds = int(max_worlds)
        self.pool_bytes = int(pool_bytes)
        h = ctypes.c_void_p()
        s = torch.cuda.current_stream() if stream is None else stream
        check(lib().sim_batch_create(self.max_worlds, _ptr(self.pool), self.pool.numel(),
                                     ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self._staged = {}

    @staticmethod
    def world_bytes(params: sim.Params, n_fil: int, n_part: int) -> int:
        cp = params.c()
        b = ctypes.c_size_t()
        check(lib().sim_batch_world_bytes(ctypes.byref(cp), int(n_fil), int(n_part), ctypes.byref(b)))
        return int(b.value)

    def admit(self, world, params: sim.Params, steps: int, t0: int = 0) -> int:
        """Copy a workloads.World's initial state into the pool; returns the slot."""
        st = sim.DeviceState(world, self.device)
        arr = st.arrays()
        cp = params.c()
        slot = ctypes.c_int32()
        check(lib().sim_batch_admit(self.handle, ctypes.byref(cp), ctypes.byref(arr), int(t0), int(steps),
                                    ctypes.byref(slot)))
        # the copies out of the staging tensors are ordered on the stream
        # before any later use of their memory; keep them until the next chunk
        self._staged[slot.value] = st
        return slot.value

    def advance(self, n_steps: int):
        check(lib().sim_batch_advance(self.handle, int(n_steps)))
        self._staged.clear()

    def remaining(self, slot: int) -> int:
        r = ctypes.c_int32()
        check(lib().sim_batch_remaining(self.handle, int(slot), ctypes.byref(r)))
        return int(r.value)

    def retire(self, slot: int, world) -> sim.DeviceState:
        """Copy a slot's state into fresh device tensors and free the slot.

        Raises SimError(SIM_E_UNSTABLE) (after freeing) if the world was flagged."""
        out = sim.DeviceState(world, self.device)
        arr = out.arrays()
        self._staged.pop(slot, None)
        check(lib().sim_batch_retire(self.handle, int(slot), ctypes.byref(arr)))
        return out

    def set_tuning(self, chunk_steps: int, cell_blocks: int, node_blocks: int):
        check(lib().sim_batch_set_tuning(self.handle, int(chunk_steps), int(cell_blocks), int(node_blocks)))

    def sync(self):
        check(lib().sim_batch_sync(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            lib().sim_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
