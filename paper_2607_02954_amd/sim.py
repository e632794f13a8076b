"""Python binding of libmicrocosm (ctypes; argument marshalling only).

Every step of the method runs in the library's HIP kernels.  Torch provides
device memory (state, workspace, pools, checkpoints) and the stream; nothing
here computes physics.  If the shared library is missing the binding raises:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmicrocosm.so")

SIM_OK, SIM_E_INVALID, SIM_E_WORKSPACE, SIM_E_HIP, SIM_E_UNSTABLE, SIM_E_STATE, SIM_E_FULL = range(7)
SIM_SPLAT_SORTED = 1
SIM_SPLAT_DIRECT = 2

# D2Q9 weights in the library's velocity order; the library stores f - w.
LATTICE_WEIGHTS = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)

EXPORTS = [
    "sim_params_default", "sim_workspace_size", "sim_create", "sim_set_workspace_size", "sim_create_set",
    "sim_step", "sim_rollout",
    "sim_checkpoint_size", "sim_backward_workspace_size", "sim_backward", "sim_sync",
    "sim_clear_flags", "sim_destroy", "sim_last_error", "sim_debug_substep", "sim_debug_buffer",
    "sim_profile_steps", "sim_measure_atomics", "sim_step_noalloc", "sim_debug_adjoint",
    "sim_density_loss_workspace_size", "sim_density_loss", "sim_rest_effort", "sim_energy_packets",
    "sim_batch_world_bytes", "sim_batch_create", "sim_batch_admit", "sim_batch_advance",
    "sim_batch_remaining", "sim_batch_retire", "sim_batch_sync", "sim_batch_set_tuning",
    "sim_batch_destroy",
]


class SimError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class SimParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("tau", ctypes.c_float), ("trt_magic", ctypes.c_float),
        ("k_bend", ctypes.c_float), ("k_stretch", ctypes.c_float), ("k_shear", ctypes.c_float),
        ("pbd_iters", ctypes.c_int32),
        ("k_elastic", ctypes.c_float), ("k_repulse", ctypes.c_float),
        ("sigma_repulse", ctypes.c_float), ("repulse_radius", ctypes.c_int32),
        ("u_max", ctypes.c_float), ("flags", ctypes.c_uint32), ("tile_side", ctypes.c_int32),
        ("energy_rate", ctypes.c_float), ("mdf_iters", ctypes.c_int32), ("marker_offset", ctypes.c_float),
    ]


class SimArrays(ctypes.Structure):
    _fields_ = [
        ("n_filaments", ctypes.c_int32), ("n_particles", ctypes.c_int32),
        ("fil_offset", ctypes.c_void_p), ("cell", ctypes.c_void_p), ("frac", ctypes.c_void_p),
        ("rest_angle", ctypes.c_void_p), ("rest_length", ctypes.c_void_p),
        ("act_amp", ctypes.c_void_p), ("act_period", ctypes.c_void_p), ("act_phase", ctypes.c_void_p),
        ("f", ctypes.c_void_p), ("u", ctypes.c_void_p),
        ("k_bend", ctypes.c_void_p), ("k_stretch", ctypes.c_void_p), ("k_shear", ctypes.c_void_p),
        ("fil_flags", ctypes.c_void_p),
        ("energy", ctypes.c_void_p), ("energy_sensed", ctypes.c_void_p), ("energy_collected", ctypes.c_void_p),
        ("fil_parent", ctypes.c_void_p), ("fil_attach", ctypes.c_void_p),
    ]


class SimSplatImage(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("sigma", ctypes.c_float), ("amp", ctypes.c_float)]


_lib = None


def lib():
    """Load libmicrocosm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_02954_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "sim_params_default": (None, [P(SimParams), i32, i32]),
        "sim_workspace_size": (i32, [P(SimParams), i32, i32, P(sz)]),
        "sim_create": (i32, [P(SimParams), P(SimArrays), vp, sz, vp, P(vp)]),
        "sim_set_workspace_size": (i32, [P(SimParams), i32, P(SimArrays), P(sz)]),
        "sim_create_set": (i32, [P(SimParams), i32, P(SimArrays), vp, sz, vp, P(vp)]),
        "sim_step": (i32, [vp, i64]),
        "sim_rollout": (i32, [vp, i64, i32, i32, vp, sz]),
        "sim_checkpoint_size": (i32, [vp, i32, i32, P(sz)]),
        "sim_backward_workspace_size": (i32, [vp, i32, P(sz)]),
        "sim_backward": (i32, [vp, i64, i32, i32, vp, vp, vp, vp, vp, sz]),
        "sim_sync": (i32, [vp]),
        "sim_clear_flags": (i32, [vp]),
        "sim_destroy": (None, [vp]),
        "sim_last_error": (ctypes.c_char_p, []),
        "sim_debug_substep": (i32, [vp, i32, i64]),
        "sim_debug_buffer": (i32, [vp, i32, P(vp)]),
        "sim_debug_adjoint": (i32, [vp, i32, vp, vp, vp]),
        "sim_profile_steps": (i32, [vp, i64, i32, P(ctypes.c_float)]),
        "sim_measure_atomics": (i32, [vp, sz, vp, P(ctypes.c_double)]),
        "sim_step_noalloc": (i32, [P(SimParams), P(SimArrays), i64, vp, vp]),
        "sim_density_loss_workspace_size": (i32, [P(SimSplatImage), P(sz)]),
        "sim_density_loss": (i32, [P(SimSplatImage), i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "sim_rest_effort": (i32, [i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "sim_energy_packets": (i32, [i32, i32, i32, vp, vp, vp, vp, vp]),
        "sim_batch_world_bytes": (i32, [P(SimParams), i32, i32, P(sz)]),
        "sim_batch_create": (i32, [i32, vp, sz, vp, P(vp)]),
        "sim_batch_admit": (i32, [vp, P(SimParams), P(SimArrays), i64, i32, P(i32)]),
        "sim_batch_advance": (i32, [vp, i32]),
        "sim_batch_remaining": (i32, [vp, i32, P(i32)]),
        "sim_batch_retire": (i32, [vp, i32, P(SimArrays)]),
        "sim_batch_sync": (i32, [vp]),
        "sim_batch_set_tuning": (i32, [vp, i32, i32, i32]),
        "sim_batch_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int):
    if status != SIM_OK:
        raise SimError(status, lib().sim_last_error().decode())


@dataclass
class Params:
    """Python mirror of sim_params (defaults equal sim_params_default)."""

    nx: int
    ny: int
    tau: float = 1.0
    trt_magic: float = 0.25
    k_bend: float = 0.5
    k_stretch: float = 1.0
    k_shear: float = 0.5
    pbd_iters: int = 4
    k_elastic: float = 0.05
    k_repulse: float = 0.1
    sigma_repulse: float = 1.0
    repulse_radius: int = 4
    u_max: float = 0.3
    transfer: str = "binned"          # "binned" (default), "sorted" or "direct"
    tile: int = 32                    # grid tile side of the tile kernels: 16, 32 or 64
    energy_rate: float = 0.0          # energy field collection rate (0: no field)
    mdf_iters: int = 1                # multi-direct forcing iterations (binned or direct transfer)
    marker_offset: float = 0.0        # two-layer marker offset in cells (binned or direct transfer)

    def flags(self) -> int:
        return {"binned": 0, "sorted": SIM_SPLAT_SORTED, "direct": SIM_SPLAT_DIRECT}[self.transfer]

    def c(self) -> SimParams:
        return SimParams(self.nx, self.ny, self.tau, self.trt_magic, self.k_bend, self.k_stretch,
                         self.k_shear, self.pbd_iters, self.k_elastic, self.k_repulse,
                         self.sigma_repulse, self.repulse_radius, self.u_max,
                         self.flags(), self.tile, self.energy_rate, self.mdf_iters, self.marker_offset)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class DeviceState:
    """Device tensors of one world's inputs and state (filament-contiguous SoA)."""

    def __init__(self, w, device="cuda"):
        dev = torch.device(device)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)
        self.nx, self.ny = int(w.nx), int(w.ny)
        self.n_fil, self.n_part = int(w.n_filaments), int(w.n_particles)
        self.fil_offset = t(w.fil_offset, torch.int32)
        self.cell = t(w.cell, torch.int32).reshape(2, -1).contiguous()
        self.frac = t(w.frac, torch.float32).reshape(2, -1).contiguous()
        self.rest_angle = t(w.rest_angle, torch.float32)
        self.rest_length = t(w.rest_length, torch.float32)
        self.act_amp = t(w.act_amp, torch.float32)
        self.act_period = t(w.act_period, torch.float32)
        self.act_phase = t(w.act_phase, torch.float32)
        self.f = torch.zeros(9, self.ny, self.nx, device=dev, dtype=torch.float32)   # fluid at rest
        self.u = torch.zeros(self.ny, self.nx, 2, device=dev, dtype=torch.float32)
        st = getattr(w, "stiffness", None)
        self.k_bend, self.k_stretch, self.k_shear = ((None,) * 3 if st is None else
                                                     tuple(t(k, torch.float32) for k in st))
        closed = getattr(w, "closed", None)
        self.fil_flags = None if closed is None else t(np.asarray(closed, dtype=np.int32), torch.int32)
        par = getattr(w, "parent", None)
        self.fil_parent = None if par is None else t(np.asarray(par, dtype=np.int32), torch.int32)
        self.fil_attach = None if par is None else t(np.asarray(w.attach, dtype=np.float32), torch.float32).contiguous()
        E = getattr(w, "energy", None)
        self.energy = None if E is None else t(E, torch.float32).reshape(self.ny, self.nx).contiguous()
        self.energy_sensed = None if E is None else torch.zeros(self.n_part, device=dev, dtype=torch.float32)
        self.energy_collected = None if E is None else torch.zeros(self.n_fil, device=dev, dtype=torch.float32)

    def arrays(self) -> SimArrays:
        return SimArrays(self.n_fil, self.n_part, _ptr(self.fil_offset), _ptr(self.cell), _ptr(self.frac),
                         _ptr(self.rest_angle), _ptr(self.rest_length), _ptr(self.act_amp),
                         _ptr(self.act_period), _ptr(self.act_phase), _ptr(self.f), _ptr(self.u),
                         _ptr(self.k_bend), _ptr(self.k_stretch), _ptr(self.k_shear), _ptr(self.fil_flags),
                         _ptr(self.energy), _ptr(self.energy_sensed), _ptr(self.energy_collected),
                         _ptr(self.fil_parent), _ptr(self.fil_attach))

    def positions64(self) -> np.ndarray:
        return self.cell.cpu().numpy().astype(np.float64) + self.frac.cpu().numpy().astype(np.float64)

    def velocity64(self) -> np.ndarray:
        """u as float64 [2, ny, nx] (the library stores it interleaved)."""
        return self.u.permute(2, 0, 1).cpu().numpy().astype(np.float64)

    def populations64(self) -> np.ndarray:
        return self.f.cpu().numpy().astype(np.float64) + LATTICE_WEIGHTS.reshape(9, 1, 1)


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def measure_atomics(device="cuda"):
    """Atomic-add throughput of the device (see sim_measure_atomics)."""
    buf = torch.empty(64 << 20, dtype=torch.uint8, device=device)
    out = (ctypes.c_double * 7)()
    check(lib().sim_measure_atomics(_ptr(buf), buf.numel(), _stream_handle(), out))
    keys = ["lds_f32_add_returned", "lds_f32_add", "lds_u64_add", "lds_u32_add"]
    res = {k: out[i] for i, k in enumerate(keys)}
    res["unit"] = "lane-ops per clock per compute unit"
    res["global_f32_atomic_per_clock_chip"] = out[4]
    res["clock_hz"] = out[5]
    res["compute_units"] = int(out[6])
    return res


def step_noalloc(state: "DeviceState", params: "Params", t: int, status: Optional[torch.Tensor] = None,
                 stream=None):
    """One step of the world held in `state` through sim_step_noalloc (no
    handle, no workspace: the library's static device scratch).  `status`,
    if given, is a device int32 tensor that receives the step's status."""
    cp = params.c()
    arr = state.arrays()
    if status is not None:
        assert status.dtype == torch.int32 and status.is_cuda
    check(lib().sim_step_noalloc(ctypes.byref(cp), ctypes.byref(arr), int(t), _ptr(status), _stream_handle(stream)))


class World:
    """A single world: caller-owned device state plus the library handle."""

    def __init__(self, w, params: Optional[Params] = None, device="cuda", stream=None):
        L = lib()
        self.params = params or Params(nx=w.nx, ny=w.ny)
        self.state = DeviceState(w, device)
        self.stream = stream
        cp = self.params.c()
        nbytes = ctypes.c_size_t()
        check(L.sim_workspace_size(ctypes.byref(cp), self.state.n_fil, self.state.n_part, ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=device)
        self._arrays = self.state.arrays()
        h = ctypes.c_void_p()
        check(L.sim_create(ctypes.byref(cp), ctypes.byref(self._arrays), _ptr(self.workspace),
                           self.workspace.numel(), _stream_handle(stream), ctypes.byref(h)))
        self.handle = h

    def step(self, t: int):
        check(lib().sim_step(self.handle, int(t)))

    def rollout(self, t0: int, n: int, ckpt_every: int = 0, ckpt: Optional[torch.Tensor] = None):
        check(lib().sim_rollout(self.handle, int(t0), int(n), int(ckpt_every), _ptr(ckpt),
                                0 if ckpt is None else ckpt.numel() * ckpt.element_size()))

    def checkpoint_bytes(self, n: int, ckpt_every: int) -> int:
        b = ctypes.c_size_t()
        check(lib().sim_checkpoint_size(self.handle, int(n), int(ckpt_every), ctypes.byref(b)))
        return int(b.value)

    def sync(self):
        check(lib().sim_sync(self.handle))

    def profile(self, t0: int, n: int):
        """Mean ms per kernel group over n real steps (see sim_profile_steps)."""
        out = (ctypes.c_float * 6)()
        check(lib().sim_profile_steps(self.handle, int(t0), int(n), out))
        return list(out)

    def substep(self, which: int, t: int):
        check(lib().sim_debug_substep(self.handle, int(which), int(t)))

    def adjoint_substep(self, which: int, x: torch.Tensor, out: torch.Tensor,
                        scratch: Optional[torch.Tensor] = None):
        """One linear adjoint sub-step (see sim_debug_adjoint), for tests."""
        check(lib().sim_debug_adjoint(self.handle, int(which), _ptr(x), _ptr(out), _ptr(scratch)))

    def buffer_view(self, which: int, shape, dtype=torch.float32) -> torch.Tensor:
        """A torch view (no copy) of an internal per-step buffer, for tests."""
        p = ctypes.c_void_p()
        check(lib().sim_debug_buffer(self.handle, int(which), ctypes.byref(p)))
        n = int(np.prod(shape))
        size = n * torch.empty(0, dtype=dtype).element_size()
        off = p.value - self.workspace.data_ptr()
        assert 0 <= off and off + size <= self.workspace.numel()
        return self.workspace[off:off + size].view(dtype).reshape(shape)

    def buffer(self, which: int, shape, dtype=torch.float32) -> torch.Tensor:
        """A copy of an internal per-step buffer, for tests."""
        return self.buffer_view(which, shape, dtype).clone()

    def close(self):
        if getattr(self, "handle", None):
            lib().sim_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _world_backward(self, t0: int, n: int, ckpt_every: int, ckpt: torch.Tensor, g_pos: torch.Tensor,
                    g_rest: torch.Tensor, g_pos0: Optional[torch.Tensor] = None):
    """dL/d(rest angle) (accumulated into g_rest) and optionally dL/dx_t0 (into
    g_pos0) of a rollout recorded with checkpoints, given g_pos = dL/dx_T."""
    L = lib()
    nb = ctypes.c_size_t()
    check(L.sim_backward_workspace_size(self.handle, int(ckpt_every), ctypes.byref(nb)))
    ws = getattr(self, "_adj_ws", None)
    if ws is None or ws.numel() < nb.value:
        ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.workspace.device)
        self._adj_ws = ws
    assert g_pos.dtype == torch.float32 and g_pos.is_contiguous() and g_pos.numel() == 2 * self.state.n_part
    assert g_rest.dtype == torch.float32 and g_rest.is_contiguous() and g_rest.numel() == self.state.n_part
    check(L.sim_backward(self.handle, int(t0), int(n), int(ckpt_every), _ptr(ckpt), _ptr(g_pos), _ptr(g_rest),
                         _ptr(g_pos0), _ptr(ws), ws.numel()))


def _positions(self) -> torch.Tensor:
    """Node positions as a float64 device tensor [2, N] (cell + frac)."""
    return self.state.cell.double() + self.state.frac.double()


World.backward = _world_backward
World.positions = _positions


class WorldSet:
    """Worlds with the same parameters stepped together in the same kernel
    launches (sim_create_set), each with its own device state.  Node vectors
    (positions, gradients) are the worlds' blocks one after another: world
    w's [2][N_w] block (or [N_w] for per-node scalars) follows world w-1's."""

    def __init__(self, worlds, params: Optional[Params] = None, device="cuda", stream=None):
        L = lib()
        self.params = params or Params(nx=worlds[0].nx, ny=worlds[0].ny)
        self.states = [DeviceState(w, device) for w in worlds]
        self.stream = stream
        self.n_parts = [st.n_part for st in self.states]
        cp = self.params.c()
        n = len(self.states)
        self._arrays = (SimArrays * n)(*[st.arrays() for st in self.states])
        nbytes = ctypes.c_size_t()
        check(L.sim_set_workspace_size(ctypes.byref(cp), n, self._arrays, ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(L.sim_create_set(ctypes.byref(cp), n, self._arrays, _ptr(self.workspace), self.workspace.numel(),
                               _stream_handle(stream), ctypes.byref(h)))
        self.handle = h

    step = World.step
    rollout = World.rollout
    checkpoint_bytes = World.checkpoint_bytes
    sync = World.sync
    close = World.close
    __del__ = World.__del__

    def positions(self) -> torch.Tensor:
        """Node positions of every world as float64, the worlds' [2][N_w] blocks in order."""
        return torch.cat([(st.cell.double() + st.frac.double()).reshape(-1) for st in self.states])

    def set_rest_angles(self, rest: torch.Tensor):
        """Write the worlds' rest angles from one array of their [N_w] blocks."""
        off = 0
        for st, n in zip(self.states, self.n_parts):
            st.rest_angle.copy_(rest[off:off + n])
            off += n

    def rest_angles(self) -> torch.Tensor:
        return torch.cat([st.rest_angle for st in self.states])

    def backward(self, t0: int, n: int, ckpt_every: int, ckpt: torch.Tensor, g_pos: torch.Tensor,
                 g_rest: torch.Tensor, g_pos0: Optional[torch.Tensor] = None):
        """sim_backward over every world of the set (blocks as in positions)."""
        L = lib()
        nb = ctypes.c_size_t()
        check(L.sim_backward_workspace_size(self.handle, int(ckpt_every), ctypes.byref(nb)))
        ws = getattr(self, "_adj_ws", None)
        if ws is None or ws.numel() < nb.value:
            ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.workspace.device)
            self._adj_ws = ws
        total = sum(self.n_parts)
        assert g_pos.dtype == torch.float32 and g_pos.is_contiguous() and g_pos.numel() == 2 * total
        assert g_rest.dtype == torch.float32 and g_rest.is_contiguous() and g_rest.numel() == total
        check(L.sim_backward(self.handle, int(t0), int(n), int(ckpt_every), _ptr(ckpt), _ptr(g_pos), _ptr(g_rest),
                             _ptr(g_pos0), _ptr(ws), ws.numel()))


class SetRollout(torch.autograd.Function):
    """The final positions of every world of a WorldSet after n_steps, as a
    function of all their rest angles (both as the worlds' blocks in order),
    differentiable through one sim_backward over the whole set."""

    @staticmethod
    def forward(ctx, rest_angles, wset, t0, n_steps, ckpt_every):
        if wset.params.transfer != "binned":
            raise SimError(SIM_E_INVALID, "differentiation needs the tile-binned transfer "
                                          f"(set uses '{wset.params.transfer}')")
        ra32 = rest_angles.detach().to(torch.float32).contiguous()
        with torch.no_grad():
            wset.set_rest_angles(ra32)
        ckpt = torch.empty(wset.checkpoint_bytes(n_steps, ckpt_every), dtype=torch.uint8,
                           device=wset.workspace.device)
        wset.rollout(t0, n_steps, ckpt_every, ckpt)
        ctx.wset, ctx.ckpt, ctx.args = wset, ckpt, (t0, n_steps, ckpt_every)
        ctx.rest = ra32.clone()
        ctx.dtype = rest_angles.dtype
        return wset.positions()

    @staticmethod
    def backward(ctx, g_x):
        t0, n, k = ctx.args
        S = ctx.wset
        g_pos = g_x.detach().to(torch.float32).contiguous()
        g_rest = torch.zeros(sum(S.n_parts), dtype=torch.float32, device=g_pos.device)
        current = S.rest_angles().clone()
        S.set_rest_angles(ctx.rest)
        try:
            S.backward(t0, n, k, ctx.ckpt, g_pos, g_rest)
        finally:
            S.set_rest_angles(current)
        return g_rest.to(ctx.dtype), None, None, None, None


class Rollout(torch.autograd.Function):
    """x_T = rollout(rest_angle) on the GPU, differentiable in the rest angles.

    Forward: copies rest_angle into the world, runs n_steps with checkpoints
    every ckpt_every steps and returns the final positions (float64 [2, N]).
    Backward: sim_backward recomputes each segment from its checkpoint and runs
    the hand-written adjoint kernels, returning dL/d(rest_angle).
    """

    @staticmethod
    def forward(ctx, rest_angle, world, t0, n_steps, ckpt_every):
        if world.params.transfer != "binned":
            # the same refusal as sim_backward's, raised before the forward runs
            raise SimError(SIM_E_INVALID, "differentiation needs the tile-binned transfer "
                                          f"(world uses '{world.params.transfer}')")
        ra32 = rest_angle.detach().to(torch.float32).contiguous()
        with torch.no_grad():
            world.state.rest_angle.copy_(ra32)
        ckpt = torch.empty(world.checkpoint_bytes(n_steps, ckpt_every), dtype=torch.uint8,
                           device=world.workspace.device)
        world.rollout(t0, n_steps, ckpt_every, ckpt)
        ctx.world, ctx.ckpt, ctx.args = world, ckpt, (t0, n_steps, ckpt_every)
        # the rest angles this forward ran with: the backward recomputes with
        # them even if the world's array has been rewritten in between
        ctx.rest = ra32.clone()
        ctx.dtype = rest_angle.dtype
        return world.positions()

    @staticmethod
    def backward(ctx, g_x):
        t0, n, k = ctx.args
        W = ctx.world
        g_pos = g_x.detach().to(torch.float32).contiguous()
        g_rest = torch.zeros(W.state.n_part, dtype=torch.float32, device=g_pos.device)
        current = W.state.rest_angle.clone()
        W.state.rest_angle.copy_(ctx.rest)
        try:
            W.backward(t0, n, k, ctx.ckpt, g_pos, g_rest)
        finally:
            W.state.rest_angle.copy_(current)        # stream-ordered after the backward
        return g_rest.to(ctx.dtype), None, None, None, None


def density_loss(nx: int, ny: int, cell: torch.Tensor, frac: torch.Tensor, target: torch.Tensor,
                 sigma: float, amp: float = 1.0, want_grad: bool = True, want_image: bool = True,
                 stream=None):
    """Folding objective of nodes at cell + frac ([2, N] int32 / float32 device
    tensors) against target ([H, W] float32 device tensor), through
    sim_density_loss.  Returns (loss device float32 [1], image [H, W] or None,
    dL/dx [2, N] float32 or None)."""
    L = lib()
    H, W = target.shape
    img = SimSplatImage(int(W), int(H), float(sigma), float(amp))
    nb = ctypes.c_size_t()
    check(L.sim_density_loss_workspace_size(ctypes.byref(img), ctypes.byref(nb)))
    dev = target.device
    ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=dev)
    N = int(cell.shape[1]) if cell.dim() == 2 else 0
    assert cell.dtype == torch.int32 and frac.dtype == torch.float32 and target.dtype == torch.float32
    assert cell.is_contiguous() and frac.is_contiguous() and target.is_contiguous()
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    image = torch.empty(H, W, dtype=torch.float32, device=dev) if want_image else None
    g_pos = torch.empty(2, N, dtype=torch.float32, device=dev) if want_grad else None
    check(L.sim_density_loss(ctypes.byref(img), int(nx), int(ny), N, _ptr(cell), _ptr(frac), _ptr(target),
                             _ptr(image), _ptr(loss), _ptr(g_pos), _ptr(ws), ws.numel(), _stream_handle(stream)))
    return loss, image, g_pos


def split_positions(x: torch.Tensor):
    """Float64 positions [2, N] as the library's (int32 cell, float32 fraction);
    exact for positions that came from (cell, fraction) pairs."""
    c = torch.floor(x)
    return c.to(torch.int32).contiguous(), (x - c).to(torch.float32).contiguous()


class DensityLoss(torch.autograd.Function):
    """L(x) = mean over pixels of (splatted density image of x - target)^2 on
    the GPU (sim_density_loss); x: float64 [2, N] positions (e.g. the output of
    Rollout), differentiable.  Chained with Rollout it gives the paper's
    folding objective's gradient in the rest angles."""

    @staticmethod
    def forward(ctx, x, nx, ny, target, sigma, amp):
        cell, frac = split_positions(x.detach())
        loss, _, g = density_loss(nx, ny, cell, frac, target, sigma, amp, want_grad=True, want_image=False)
        ctx.save_for_backward(g)
        ctx.dtype = x.dtype
        return loss[0].to(x.dtype)

    @staticmethod
    def backward(ctx, g_out):
        (g,) = ctx.saved_tensors
        return g.to(ctx.dtype) * g_out, None, None, None, None, None


def rest_effort(state: "DeviceState", new_rest_angle: torch.Tensor, new_rest_length: torch.Tensor,
                effort: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Bending and stretching effort ([2, F], accumulated into `effort`) of
    replacing the world's rest angles and lengths by the new ones
    (sim_rest_effort); the caller then writes the new values."""
    if effort is None:
        effort = torch.zeros(2, state.n_fil, dtype=torch.float32, device=state.f.device)
    for t in (new_rest_angle, new_rest_length):
        assert t.dtype == torch.float32 and t.is_contiguous() and t.numel() == state.n_part
    check(lib().sim_rest_effort(state.n_fil, _ptr(state.fil_offset), _ptr(state.fil_flags), _ptr(state.rest_angle),
                                _ptr(new_rest_angle), _ptr(state.rest_length), _ptr(new_rest_length), _ptr(effort),
                                _stream_handle(stream)))
    return effort


def energy_packets(nx: int, ny: int, centres: torch.Tensor, amps: torch.Tensor, widths: torch.Tensor,
                   field: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Add Gaussian packets (centres [2, P], amps [P], widths [P], float32
    device tensors) to a field [ny, nx] (sim_energy_packets); a new zero field
    if none is given."""
    if field is None:
        field = torch.zeros(ny, nx, dtype=torch.float32, device=centres.device)
    P = int(amps.numel())
    check(lib().sim_energy_packets(int(nx), int(ny), P, _ptr(centres.contiguous()), _ptr(amps), _ptr(widths),
                                   _ptr(field), _stream_handle(stream)))
    return field
