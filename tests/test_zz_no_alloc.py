"""sim_step_noalloc (static device scratch, no allocation) against sim_step.

Two worlds in a row, the second smaller than the first, in every transfer
mode: each call of the allocation-free entry point must give the state that
sim_create + sim_step give from the same state, to the parity bar (positions
relative 1e-5 and per-step displacement 1e-4, grid velocity 1e-4).  Also: the
status word, and offsets that fail the device-side checks leave the state
untouched.
"""
import numpy as np
import pytest
import torch

from paper_2607_02954_amd import workloads as wl
from parity_util import TOL_D, TOL_U, TOL_X, disp_err, rel

pytestmark = pytest.mark.gpu

MODES = ["binned", "sorted", "direct"]


def _sim():
    from paper_2607_02954_amd import sim
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sim


def _compare(sim, w, mode, t0, steps, status):
    p = sim.Params(nx=w.nx, ny=w.ny, transfer=mode)
    ref = sim.World(w, p)                          # sim_create + sim_step
    st = sim.DeviceState(w, "cuda")                # the same initial state
    for t in range(t0, t0 + steps):
        x_before = st.positions64()
        ref.step(t)
        status.fill_(-1)
        sim.step_noalloc(st, p, t, status)
        torch.cuda.synchronize()
        ref.sync()
        xr, xn = ref.state.positions64(), st.positions64()
        e_x = rel(xn, xr)
        e_d = disp_err(xn - x_before, xr - x_before)
        e_u = rel(st.velocity64(), ref.state.velocity64())
        e_f = rel(st.populations64(), ref.state.populations64())
        same = all(torch.equal(getattr(st, k), getattr(ref.state, k)) for k in ("cell", "frac", "f", "u"))
        print(f"noalloc {mode} {w.nx}x{w.ny} N={w.n_particles} t={t}: e_x={e_x:.2e} e_d={e_d:.2e} "
              f"e_u={e_u:.2e} e_f={e_f:.2e} bitwise={same}", flush=True)
        assert int(status.item()) == sim.SIM_OK
        assert e_x <= TOL_X and e_d <= TOL_D and e_u <= TOL_U and e_f <= TOL_U
    ref.close()


@pytest.mark.parametrize("mode", MODES)
def test_noalloc_equals_step_two_worlds(mode):
    sim = _sim()
    status = torch.empty(1, dtype=torch.int32, device="cuda")
    big = wl.random_world(3, 80, 72, [3, 1, 2, 40, 17, 64, 9, 130, 5], amp=0.5)
    small = wl.random_world(4, 64, 48, [32, 9, 20], amp=0.5)
    assert small.nx * small.ny < big.nx * big.ny and small.n_particles < big.n_particles
    _compare(sim, big, mode, 0, 2, status)
    _compare(sim, small, mode, 5, 2, status)


def test_noalloc_rejects_bad_offsets_on_device():
    sim = _sim()
    w = wl.random_world(5, 64, 48, [12, 9, 20], amp=0.5)
    p = sim.Params(nx=w.nx, ny=w.ny)
    st = sim.DeviceState(w, "cuda")
    st.fil_offset[1] = 25                           # filament 1 gets a negative length
    cell0, frac0, f0 = st.cell.clone(), st.frac.clone(), st.f.clone()
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    sim.step_noalloc(st, p, 0, status)
    torch.cuda.synchronize()
    assert int(status.item()) == sim.SIM_E_INVALID
    assert torch.equal(st.cell, cell0) and torch.equal(st.frac, frac0) and torch.equal(st.f, f0)
