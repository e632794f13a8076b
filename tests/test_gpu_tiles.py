"""Tile side of the tile kernels (16, 32 or 64 cells; sim_params.tile_side)
against the FP64 oracle and across sides.

The binned transfer sums in 64-bit fixed point and every per-cell and
per-node expression is evaluated the same way whatever the tiling, so a world
run with any tile side is bitwise the same; each side is also compared with
the oracle per step (e_x <= 1e-5, e_u <= 1e-4, per-step displacement
e_d <= 1e-4) on grids narrower than a tile, ragged grids with partial last
tiles at every radius, and a dense world whose spread lists overflow.  A batch
that mixes tile sides equals its worlds run alone, and the adjoint matches
the oracle's for each side.
"""
import numpy as np
import pytest
import torch

from paper_2607_02954_amd import workloads as wl
from parity_util import TOL_D, TOL_U, TOL_X, final_state_errors, oracle_params
from test_gpu_adjoint import _compare, _gpu_grad, _joints, _oracle_grad
from test_gpu_parity import _rollout_compare, ragged_world

pytestmark = pytest.mark.gpu

SIDES = [16, 32, 64]


def _sim():
    from paper_2607_02954_amd import sim
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sim


@pytest.mark.parametrize("tile", [16, 64])
def test_tile_side_matches_oracle(tile):
    sim = _sim()
    cases = [(ragged_world(2), 20, {}),
             (wl.random_world(7, 8, 8, [3], amp=0.5), 8, {}),
             (wl.random_world(7, 40, 24, [6, 4], amp=0.5), 8, {}),
             (wl.random_world(11, 100, 97, [30, 12, 1, 50, 8], amp=0.5), 6,
              {"repulse_radius": 8, "sigma_repulse": 2.0}),
             (wl.random_world(11, 130, 66, [25, 7, 80, 2], amp=0.5), 6,
              {"repulse_radius": 1, "sigma_repulse": 0.5}),
             (wl.random_world(11, 150, 141, [40, 3, 60, 2, 33], amp=0.5), 6,
              {"repulse_radius": 6, "sigma_repulse": 1.5}),
             (wl.random_world(13, 64, 64, [60] * 50, amp=0.5), 6, {})]      # dense: lists overflow
    for w, n, kw in cases:
        for mode in ("binned", "sorted"):
            E = _rollout_compare(sim, w, n, mode, tile=tile, **kw)
            print(f"tile {tile} {w.nx}x{w.ny} N={w.n_particles} [{mode}] {kw}: {E}")


def test_tile_sides_are_bitwise_equal():
    sim = _sim()
    worlds = [wl.uniform_population(1, n_fil=300, length=40, nx=192, ny=160),
              wl.random_world(13, 64, 64, [60] * 50, amp=0.5),
              wl.random_world(11, 100, 97, [30, 12, 1, 50, 8], amp=0.5)]
    for w in worlds:
        out = {}
        for tile in SIDES:
            W = sim.World(w, sim.Params(nx=w.nx, ny=w.ny, tile=tile))
            W.rollout(0, 30)
            W.sync()
            out[tile] = [getattr(W.state, k).cpu() for k in ("cell", "frac", "f", "u")]
            W.close()
        for tile in (16, 64):
            same = all(torch.equal(a, b) for a, b in zip(out[32], out[tile]))
            print(f"{w.nx}x{w.ny} N={w.n_particles}: tile {tile} bitwise equal to tile 32: {same}")
            assert same


def test_batch_mixing_tile_sides():
    sim = _sim()
    from paper_2607_02954_amd import batch
    worlds = [wl.random_world(20 + i, nx, ny, lens, amp=0.5)
              for i, (nx, ny, lens) in enumerate([(64, 64, [20, 9]), (96, 64, [40] * 6), (128, 128, [64] * 20),
                                                  (72, 50, [3, 1, 17]), (160, 96, [12] * 30)])]
    tiles = [16, 32, 64, 16, 64]
    steps = [30, 44, 18, 60, 26]
    eng = batch.BatchEngine(max_worlds=8, pool_bytes=256 << 20)
    slots = [eng.admit(w, sim.Params(nx=w.nx, ny=w.ny, tile=t), s) for w, t, s in zip(worlds, tiles, steps)]
    while any(eng.remaining(s) > 0 for s in slots):
        eng.advance(10)
    for w, t, sl, st in zip(worlds, tiles, slots, steps):
        got = eng.retire(sl, w)
        W = sim.World(w, sim.Params(nx=w.nx, ny=w.ny, tile=t))
        W.rollout(0, st)
        W.sync()
        assert all(torch.equal(getattr(got, k).cpu(), getattr(W.state, k).cpu()) for k in ("cell", "frac", "f", "u"))
        ex, ea, eu, ed = final_state_errors(w, got, oracle_params(sim.Params(nx=w.nx, ny=w.ny)), 0, st)
        print(f"batch tile {t} {w.nx}x{w.ny}: e_x={ex:.2e} e_a={ea:.2e} e_u={eu:.2e} e_d={ed:.2e}")
        assert ex <= TOL_X and eu <= TOL_U and ed <= TOL_D


@pytest.mark.parametrize("tile", [16, 64])
def test_adjoint_with_tile_side(tile):
    sim = _sim()
    w = wl.random_world(3, 80, 72, [12, 7, 20, 2, 30], amp=0.5)
    x0 = w.positions64()
    target = x0 + np.random.default_rng(1).normal(0, 0.5, size=x0.shape)
    g, _, W, p = _gpu_grad(sim, w, target, 12, 5, tile=tile)
    ref, _ = _oracle_grad(w, p, target, 12, 5)
    err, cos = _compare(g, ref, _joints(w))
    print(f"adjoint tile {tile}: rel err {err:.2e} cos {cos:.6f}")
    assert err <= 1e-3 and cos >= 0.9999
