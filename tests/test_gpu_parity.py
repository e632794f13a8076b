"""GPU (HIP, FP32) versus the FP64 oracle, element by element, through the C ABI.

Acceptance (per step, measured errors printed; measures in parity_util):
  e_x = max_i |x_gpu - x_ref|_inf / max_i |x_ref|_inf  <= 1e-5
  e_u = max_c |u_gpu - u_ref|_inf / max_c |u_ref|_inf  <= 1e-4
  e_d (each step's displacement, both sides from the GPU's state) <= 1e-4
and the largest absolute position error in cells is printed beside them.
Sub-steps are compared normwise with tolerances derived from FP32 rounding of
O(10)-term sums (a few 1e-7 relative), allowing for atomics' arbitrary order.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_02954_amd import workloads as wl
from parity_util import (TOL_D, TOL_U, TOL_X, abs_err, disp_err, oracle_from, oracle_params, rel,
                         state64)

pytestmark = pytest.mark.gpu

DT = torch.float64


def _sim():
    from paper_2607_02954_amd import sim
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sim


def ragged_world(seed=0):
    # lengths that straddle pack boundaries, single-node and two-node filaments,
    # a grid that is not a multiple of the filter tile
    lengths = [3, 1, 2, 40, 17, 64, 9, 130, 5]
    return wl.random_world(seed, 80, 72, lengths, amp=0.5)


def gpu_state(W):
    x = torch.from_numpy(W.state.positions64())
    f = torch.from_numpy(W.state.populations64())
    return x, f


MODES = ["binned", "sorted", "direct"]


def _mk(sim, w, mode="binned", **kw):
    p = sim.Params(nx=w.nx, ny=w.ny, transfer=mode, **kw)
    return sim.World(w, p), oracle_params(p)


@pytest.mark.parametrize("mode", MODES)
def test_substeps_match_oracle(mode):
    sim = _sim()
    w = ragged_world(1)
    W, op = _mk(sim, w, mode)
    inp = O.inputs_from_world(w)
    W.rollout(0, 6)                       # non-trivial shared state
    torch.cuda.synchronize()
    t = 6
    x, f = gpu_state(W)
    tr = {}
    O.step(x, f, t, inp, op, trace=tr)
    N, ny, nx = w.n_particles, w.ny, w.nx
    W.substep(0, t)
    fel = W.buffer(4, (2, N)).cpu().numpy()             # elastic force
    e_el = rel(fel, tr["f_el"].numpy())
    assert e_el < 2e-5, e_el
    if mode == "direct":
        s = W.buffer(0, (ny, nx)).cpu().numpy()
        assert rel(s, tr["s"].numpy()) < 1e-6
    W.substep(1, t)
    G = W.buffer(1, (ny, nx, 2)).permute(2, 0, 1).cpu().numpy()
    Gref = O.central_difference(tr["st"]).numpy()
    assert rel(G, Gref) < 1e-5
    W.substep(2, t)
    F = W.buffer(3, (2, N)).cpu().numpy()
    assert rel(F, tr["force"].numpy()) < 2e-5
    Fg = W.buffer(2, (ny, nx, 2)).permute(2, 0, 1).cpu().numpy()
    assert rel(Fg, tr["Fg"].numpy()) < 2e-5
    W.substep(3, t)
    torch.cuda.synchronize()
    u = W.state.velocity64()
    e_u = rel(u, tr["u"].numpy())
    assert e_u < TOL_U, e_u
    fref = O.lbm_stream(tr["fstar"]).numpy()
    fg = W.state.populations64()
    assert np.max(np.abs(fg - fref)) < 1e-6
    W.substep(4, t)
    torch.cuda.synchronize()
    dref = O.interpolate(x, tr["u"], op).numpy()
    xg = W.state.positions64()
    xref = x.numpy() + dref
    e_x, e_d = rel(xg, xref), disp_err(xg - x.numpy(), dref)
    assert e_x < TOL_X and e_d < TOL_D, (e_x, e_d)
    print(f"substeps[{mode}]: e_el={e_el:.2e} e_u={e_u:.2e} e_x={e_x:.2e} e_d={e_d:.2e} "
          f"(max step {np.max(np.abs(dref)):.2e} cells, abs err {abs_err(xg, xref):.2e} cells)")


class Errs:
    """Largest e_x, e_a, e_u, e_d seen over a run."""

    def __init__(self):
        self.ex = self.ea = self.eu = self.ed = 0.0

    def add(self, ex, ea, eu, ed):
        self.ex, self.ea = max(self.ex, ex), max(self.ea, ea)
        self.eu, self.ed = max(self.eu, eu), max(self.ed, ed)

    def __str__(self):
        return f"e_x={self.ex:.2e} e_a={self.ea:.2e} cells e_u={self.eu:.2e} e_d={self.ed:.2e}"


def _rollout_compare(sim, w, n, mode, report_every=0, **kw):
    """n single steps on the GPU beside the oracle's own trajectory (e_x, e_a,
    e_u at every step) and, every step, an oracle step from the GPU's state
    (e_d of that step's displacement)."""
    W, op = _mk(sim, w, mode, **kw)
    inp = O.inputs_from_world(w)
    x = O.positions_from_world(w)
    f = O.rest_populations(op)
    E = Errs()
    for t in range(n):
        xs, fs = gpu_state(W)                       # shared state of this step
        xs_next, _, _ = oracle_from(xs, fs, t, 1, inp, op)
        W.step(t)
        with torch.no_grad():
            x, f, u = O.step(x, f, t, inp, op)
        torch.cuda.synchronize()
        xg = W.state.positions64()
        ex, ea = rel(xg, x.numpy()), abs_err(xg, x.numpy())
        eu = rel(W.state.velocity64(), u.numpy())
        ed = disp_err(xg - xs.numpy(), (xs_next - xs).numpy())
        E.add(ex, ea, eu, ed)
        assert ex <= TOL_X, (t, ex)
        assert eu <= TOL_U, (t, eu)
        assert ed <= TOL_D, (t, ed)
        if report_every and (t + 1) % report_every == 0:
            print(f"  [{mode}] step {t + 1:5d}: e_x={ex:.2e} e_a={ea:.2e} cells e_u={eu:.2e} e_d={ed:.2e} "
                  f"(max so far: {E})", flush=True)
    W.sync()
    return E


@pytest.mark.parametrize("mode", MODES)
def test_single_chain_100_steps(mode):
    sim = _sim()
    E = _rollout_compare(sim, wl.parity_single(0), 100, mode)
    print(f"single chain 32 nodes 64^2, 100 steps [{mode}]: {E}")


@pytest.mark.parametrize("mode", MODES)
def test_ragged_population_100_steps(mode):
    sim = _sim()
    E = _rollout_compare(sim, ragged_world(2), 100, mode)
    print(f"ragged population, 100 steps [{mode}]: {E}")


def test_graph_rollout_equals_stepwise_and_sorted_is_deterministic():
    sim = _sim()
    w = ragged_world(3)
    runs = []
    for mode in ("rollout", "rollout", "step"):
        W, _ = _mk(sim, w, "sorted")
        if mode == "rollout":
            W.rollout(0, 37)
        else:
            for t in range(37):
                W.step(t)
        torch.cuda.synchronize()
        runs.append((W.state.cell.cpu().clone(), W.state.frac.cpu().clone(), W.state.f.cpu().clone(),
                     W.state.u.cpu().clone()))
    for a, b in zip(runs[0], runs[1]):
        assert torch.equal(a, b)            # bitwise reproducible
    for a, b in zip(runs[0], runs[2]):
        assert torch.equal(a, b)            # graph path == plain launches
    Wa, _ = _mk(sim, w, "binned")
    Wa.rollout(0, 37)
    torch.cuda.synchronize()
    xs = runs[0][0].numpy() + runs[0][1].numpy().astype(np.float64)
    assert rel(Wa.state.positions64(), xs) < TOL_X


def test_checkpoints_hold_segment_start_states():
    sim = _sim()
    w = ragged_world(4)
    W, _ = _mk(sim, w, "sorted")
    nb = W.checkpoint_bytes(30, 10)
    ck = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    W.rollout(0, 30, 10, ck)
    torch.cuda.synchronize()
    ref, _ = _mk(sim, w, "sorted")
    N = w.n_particles
    per = nb // 3
    for seg in range(3):
        blob = ck[seg * per:(seg + 1) * per]
        cell = blob[: 8 * N].view(torch.int32).reshape(2, N).cpu()
        assert torch.equal(cell, ref.state.cell.cpu())
        ref.rollout(seg * 10, 10)
        torch.cuda.synchronize()
    assert torch.equal(W.state.cell.cpu(), ref.state.cell.cpu())
    assert torch.equal(W.state.frac.cpu(), ref.state.frac.cpu())


@pytest.mark.parametrize("mode", MODES)
def test_edge_cases(mode):
    sim = _sim()
    # empty world: fluid stays at rest
    empty = wl._assemble(32, 24, [], [], [], [], [], [])
    W, _ = _mk(sim, empty, mode)
    W.rollout(0, 5)
    W.sync()
    assert float(W.state.f.abs().max()) < 1e-7
    # one long filament (> 256 nodes uses the 1024-node pack) plus single nodes
    long = wl.random_world(5, 96, 96, [600, 1, 1, 2], amp=0.5)
    E = _rollout_compare(sim, long, 10, mode)
    print(f"long filament [{mode}]: {E}")


def test_mach_guard_flags_world():
    sim = _sim()
    W, _ = _mk(sim, ragged_world(6), "binned", u_max=1e-9)
    W.rollout(0, 4)
    with pytest.raises(sim.SimError) as ei:
        W.sync()
    assert ei.value.status == sim.SIM_E_UNSTABLE


@pytest.mark.parametrize("mode", MODES)
def test_uniform_population_full_size_steps(mode):
    # 1024 chains x 64 nodes on 512^2 with active bending: every element of
    # positions and u after each of 3 steps from the shared state
    sim = _sim()
    w = wl.uniform_population(0)
    E = _rollout_compare(sim, w, 3, mode)
    print(f"uniform 65536 nodes 512^2 [{mode}]: {E}")


@pytest.mark.parametrize("mode", MODES)
def test_small_and_ragged_grids(mode):
    # grids narrower than a tile, not multiples of the tile, and wrapping
    # supports that alias inside the filter halo
    sim = _sim()
    for (nx, ny, lens) in [(8, 8, [3]), (40, 24, [6, 4]), (72, 50, [20, 1, 9])]:
        w = wl.random_world(7, nx, ny, lens, amp=0.5)
        E = _rollout_compare(sim, w, 12, mode)
        print(f"{nx}x{ny} [{mode}]: {E}")


@pytest.mark.parametrize("mode", MODES)
def test_partial_tiles_and_radii(mode):
    # four or more tiles per axis with a narrow partial last tile (a filter or
    # spread window then reaches across it into the tile beyond), with the
    # smallest and largest Gaussian radii: every bin run and padded window
    # shape of the binned transfer at a periodic seam
    sim = _sim()
    for (nx, ny, R, sig, lens) in [(100, 97, 8, 2.0, [30, 12, 1, 50, 8]),
                                   (130, 66, 1, 0.5, [25, 7, 80, 2]),
                                   (97, 129, 6, 1.5, [40, 3, 60, 2, 33])]:
        w = wl.random_world(11, nx, ny, lens, amp=0.5)
        E = _rollout_compare(sim, w, 8, mode, repulse_radius=R, sigma_repulse=sig)
        print(f"{nx}x{ny} R={R} [{mode}]: {E}")


@pytest.mark.parametrize("mode", MODES)
def test_dense_world(mode):
    # about 0.73 nodes per cell: a tile's spread list (nodes with homes in a
    # 35 x 35 cell square) then holds 629 to 1116 nodes at the first step, so
    # one tile exceeds the 1024-record list the filter fills for the spread
    # and reads the bins instead, beside tiles that use their list (one of
    # them one record short of the limit)
    sim = _sim()
    w = wl.random_world(13, 64, 64, [60] * 50, amp=0.5)
    if mode == "binned":
        # the first step's lists: nodes whose home cell lies in
        # [x0 - 2, x0 + 32] x [y0 - 2, y0 + 32] (periodic) of each 32 x 32 tile
        x = w.positions64()
        hx, hy = np.floor(x[0]).astype(int) % 64, np.floor(x[1]).astype(int) % 64
        per_tile = [int(((((hx - x0 + 2) % 64) <= 34) & (((hy - y0 + 2) % 64) <= 34)).sum())
                    for y0 in (0, 32) for x0 in (0, 32)]
        assert max(per_tile) > 1024 and min(per_tile) <= 1024, per_tile
    E = _rollout_compare(sim, w, 6, mode)
    print(f"dense 3000 nodes 64x64 [{mode}]: {E}")


@pytest.mark.parametrize("mode", MODES)
def test_scaling_workload_full_size(mode):
    # the benchmark's million-node workload at full size: every node and cell.
    # The tile-binned transfer (the benchmark's) runs one captured 20-step
    # chunk graph, the launch configuration the benchmark times; the two
    # reference transfers run two steps.  Positions, u of the last step, and
    # the displacement over the run from the shared initial state.
    sim = _sim()
    w = wl.scaling_population(0)
    n = 20 if mode == "binned" else 2
    W, op = _mk(sim, w, mode)
    W.rollout(0, n)
    W.sync()
    inp = O.inputs_from_world(w)
    x0 = O.positions_from_world(w)
    x, _, u = oracle_from(x0, O.rest_populations(op), 0, n, inp, op)
    xg = W.state.positions64()
    ex, ea = rel(xg, x.numpy()), abs_err(xg, x.numpy())
    eu = rel(W.state.velocity64(), u.numpy())
    ed = disp_err(xg - x0.numpy(), (x - x0).numpy())
    print(f"scaling 1M nodes 2048^2, {n} steps [{mode}]: e_x={ex:.2e} e_a={ea:.2e} cells e_u={eu:.2e} "
          f"e_d={ed:.2e} (max displacement {float((x - x0).abs().max()):.2e} cells)")
    assert ex <= TOL_X and eu <= TOL_U and ed <= TOL_D


@pytest.mark.parametrize("mode", MODES)
def test_parity_config_1000_steps(mode):
    # the parity configuration in full: one 32-node chain on 64^2, 1000 steps,
    # per-step errors asserted and the error growth printed every 100 steps
    sim = _sim()
    E = _rollout_compare(sim, wl.parity_single(0), 1000, mode, report_every=100)
    print(f"single chain 32 nodes 64^2, 1000 steps [{mode}]: {E}")


def test_binned_transfer_is_bitwise_reproducible():
    # the binned transfer sums in 64-bit fixed point, so the order in which
    # nodes land in their bins cannot change any result
    sim = _sim()
    w = wl.uniform_population(1, n_fil=300, length=40, nx=192, ny=160)
    out = []
    for _ in range(2):
        W, _ = _mk(sim, w, "binned")
        W.rollout(0, 40)
        torch.cuda.synchronize()
        out.append((W.state.cell.cpu(), W.state.frac.cpu(), W.state.f.cpu(), W.state.u.cpu()))
    for a, b in zip(*out):
        assert torch.equal(a, b)
