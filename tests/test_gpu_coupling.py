"""Coupling leakage fixes on the GPU against the FP64 oracle (Methods,
Fluid-filament Interaction: Multi-Direct Forcing; the filament broadcast as a
two-layer version of itself): MDF and two layers on the direct and the
tile-binned transfer.

Per step: e_x <= 1e-5, e_u <= 1e-4 and each step's displacement e_d <= 1e-4
from the GPU's state, for one and two layers, one to eight MDF iterations,
every tile side, chains and loops, and grids smaller than a tile's windows
(which wrap onto themselves); the combinations that are not built are
refused (MDF or two layers on the sorted transfer, the adjoint off the
binned transfer); the allocation-free step and batches
mixing direct, binned, one- and two-layer MDF worlds give the single
world's results (to the parity bar: the direct transfer sums with float
atomics).
"""
import numpy as np
import pytest
import torch

from paper_2607_02954_amd import workloads as wl
from parity_util import TOL_D, TOL_U, TOL_X, disp_err, final_state_errors, oracle_params, rel
from test_gpu_parity import _rollout_compare, ragged_world

pytestmark = pytest.mark.gpu


def _sim():
    from paper_2607_02954_amd import sim
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sim


@pytest.mark.parametrize("mode,mdf,offset,tile", [("direct", 1, 0.5, 32), ("direct", 4, 0.0, 32),
                                                  ("direct", 4, 0.5, 32), ("direct", 8, 1.0, 32),
                                                  ("binned", 4, 0.0, 32), ("binned", 8, 0.0, 16),
                                                  ("binned", 3, 0.0, 64), ("binned", 1, 0.5, 32),
                                                  ("binned", 4, 0.5, 32), ("binned", 8, 1.0, 16),
                                                  ("binned", 3, 0.7, 64), ("binned", 1, 1.0, 64)])
def test_mdf_and_two_layers_match_oracle(mode, mdf, offset, tile):
    sim = _sim()
    worlds = [(ragged_world(2), 15), (wl.generality_world(3, 72, 64, [20, 2, 1], [9, 10]), 10)]
    if offset > 0.0:
        # windows that wrap onto themselves along y (and, for the markers'
        # wider node range, along x as well with 32-cell tiles)
        worlds.append((wl.random_world(4, 36, 30, [12, 9, 1], amp=0.5), 10))
    for w, n in worlds:
        E = _rollout_compare(sim, w, n, mode, mdf_iters=mdf, marker_offset=offset, tile=tile)
        print(f"MDF {mdf}, offset {offset} [{mode}, tile {tile}], {w.nx}x{w.ny} N={w.n_particles}: {E}")


@pytest.mark.parametrize("mode,mdf", [("binned", 1), ("binned", 3), ("direct", 1)])
def test_two_layers_on_branched_creatures(mode, mdf):
    # the markers' normals come from each filament's own neighbours (an
    # attachment edge is not a tangent); children and parents, chains and
    # loops, on both transfers and with MDF
    sim = _sim()
    w = wl.branched_world(5, 72, 64, 3)
    E = _rollout_compare(sim, w, 10, mode, mdf_iters=mdf, marker_offset=0.5)
    print(f"branched creatures, two layers, MDF {mdf} [{mode}], N={w.n_particles}: {E}")


@pytest.mark.parametrize("mode", ["binned", "direct"])
def test_edge_cases_with_mdf_and_two_layers(mode):
    sim = _sim()
    # an empty world stays at rest; a world of single nodes and two-node
    # filaments (no tangent beyond their one edge) and a filament longer than
    # 256 nodes (the 1024-node pack) match the oracle
    empty = wl._assemble(32, 24, [], [], [], [], [], [])
    W = sim.World(empty, sim.Params(nx=32, ny=24, transfer=mode, mdf_iters=3, marker_offset=0.5))
    W.rollout(0, 5)
    W.sync()
    assert float(W.state.f.abs().max()) < 1e-7
    W.close()
    for w in (wl.random_world(6, 48, 40, [1, 2, 1, 2, 1], amp=0.5), wl.random_world(7, 96, 96, [600, 3], amp=0.5)):
        E = _rollout_compare(sim, w, 8, mode, mdf_iters=3, marker_offset=0.5)
        print(f"MDF 3, two layers [{mode}], {w.nx}x{w.ny} N={w.n_particles}: {E}")


def test_unbuilt_combinations_are_refused():
    sim = _sim()
    w = ragged_world(1)
    for mode, kw in (("sorted", {"mdf_iters": 3}), ("sorted", {"marker_offset": 0.5}),
                     ("sorted", {"mdf_iters": 3, "marker_offset": 0.5}), ("binned", {"marker_offset": 1.5})):
        with pytest.raises(sim.SimError) as ei:
            sim.World(w, sim.Params(nx=w.nx, ny=w.ny, transfer=mode, **kw))
        assert ei.value.status == sim.SIM_E_INVALID
    # the adjoint takes MDF and two layers on the binned transfer only
    for mode, kw in (("direct", {"mdf_iters": 3}), ("direct", {"marker_offset": 0.5})):
        W = sim.World(w, sim.Params(nx=w.nx, ny=w.ny, transfer=mode, **kw))
        ra = torch.tensor(w.rest_angle, dtype=torch.float64, device="cuda", requires_grad=True)
        with pytest.raises(sim.SimError) as ei:
            sim.Rollout.apply(ra, W, 0, 4, 2).sum().backward()
        assert ei.value.status == sim.SIM_E_INVALID
        W.close()


def _close(sim, a, b, x_before):
    xa, xb = a.positions64(), b.positions64()
    return (rel(xa, xb), disp_err(xa - x_before, xb - x_before), rel(a.velocity64(), b.velocity64()))


@pytest.mark.parametrize("mode", ["direct", "binned"])
def test_noalloc_with_mdf_and_two_layers(mode):
    sim = _sim()
    w = wl.random_world(5, 80, 64, [20, 9, 33], amp=0.5)
    p = sim.Params(nx=w.nx, ny=w.ny, transfer=mode, mdf_iters=4, marker_offset=0.5)
    ref = sim.World(w, p)
    st = sim.DeviceState(w, "cuda")
    status = torch.empty(1, dtype=torch.int32, device="cuda")
    for t in range(4):
        x0 = st.positions64()
        ref.step(t)
        sim.step_noalloc(st, p, t, status)
        torch.cuda.synchronize()
        ex, ed, eu = _close(sim, st, ref.state, x0)
        print(f"noalloc {mode} MDF 4, two layers, t={t}: e_x={ex:.2e} e_d={ed:.2e} e_u={eu:.2e}")
        assert int(status.item()) == sim.SIM_OK and ex <= TOL_X and ed <= TOL_D and eu <= TOL_U, (t, ex, ed, eu)


def test_batch_with_mdf_and_two_layers():
    sim = _sim()
    from paper_2607_02954_amd import batch
    w = wl.random_world(5, 80, 64, [20, 9, 33], amp=0.5)
    worlds = [w, wl.generality_world(6, 64, 64, [15], [11]), wl.random_world(7, 72, 56, [12, 30], amp=0.5),
              wl.random_world(8, 64, 48, [25, 7], amp=0.5), wl.generality_world(9, 48, 40, [10], [12])]
    steps = [20, 14, 16, 12, 18]
    kws = [dict(transfer="direct", mdf_iters=4, marker_offset=0.5), dict(transfer="direct", mdf_iters=4, marker_offset=0.5),
           dict(transfer="binned", mdf_iters=5), dict(transfer="binned", mdf_iters=3, marker_offset=0.5),
           dict(transfer="binned", marker_offset=1.0)]
    eng = batch.BatchEngine(max_worlds=5, pool_bytes=96 << 20)
    slots = [eng.admit(x, sim.Params(nx=x.nx, ny=x.ny, **kw), s) for x, s, kw in zip(worlds, steps, kws)]
    while any(eng.remaining(s) > 0 for s in slots):
        eng.advance(10)
    for x, sl, s, kw in zip(worlds, slots, steps, kws):
        got = eng.retire(sl, x)
        op = oracle_params(sim.Params(nx=x.nx, ny=x.ny, mdf_iters=kw.get("mdf_iters", 1), marker_offset=kw.get("marker_offset", 0.0)))
        ex, ea, eu, ed = final_state_errors(x, got, op, 0, s)
        print(f"batched MDF world {x.nx}x{x.ny}, {s} steps vs oracle: e_x={ex:.2e} e_u={eu:.2e} e_d={ed:.2e}")
        assert ex <= TOL_X and eu <= TOL_U and ed <= TOL_D
