"""The paper's extensions at the sizes and in the launch configuration the
benchmark times them (2048^2 grid, 32-cell tiles, binned transfer), against
the FP64 oracle over two steps from the same initial world: e_x <= 1e-5,
e_u <= 1e-4 and the displacement e_d <= 1e-4.

  * multi-direct forcing (4 iterations) on two-layer markers, 262,144 nodes
    (Methods, Fluid-filament Interaction);
  * the energy field on the million-node workload (Methods, Fields): the
    field, each node's sensed value and each filament's collection after the
    two steps (relative max-norm <= 1e-5); the initial field is the oracle's
    own sum of 64 seeded Gaussian packets;
  * about a million nodes of branched creatures (Methods, Filaments: loops
    and branches).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_02954_amd import workloads as wl
from parity_util import TOL_D, TOL_U, TOL_X, final_state_errors, oracle_params, rel

pytestmark = pytest.mark.gpu
DT = torch.float64
TOL_E = 1e-5


def _sim():
    from paper_2607_02954_amd import sim
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sim


@pytest.mark.parametrize("case", ["mdf4_two_layers_262144", "energy_1048576", "branched_about_1M"])
def test_extension_rows_full_size(case):
    sim = _sim()
    n = 2
    if case.startswith("mdf4"):
        w = wl.random_world(0, 2048, 2048, wl.scaling_lengths(0, 1_048_576 // 4), amp=0.5)
        p = sim.Params(nx=2048, ny=2048, tile=32, mdf_iters=4, marker_offset=0.5)
    elif case.startswith("energy"):
        w = wl.scaling_population(0)
        g = np.random.default_rng(23)
        c = torch.tensor(g.uniform(0.0, 2048.0, size=(2, 64)), dtype=DT)
        a = torch.tensor(g.uniform(0.5, 2.0, size=64), dtype=DT)
        s = torch.tensor(g.uniform(50.0, 200.0, size=64), dtype=DT)
        E0 = O.energy_packets(2048, 2048, c, a, s)
        w.energy = E0.numpy().astype(np.float32)
        p = sim.Params(nx=2048, ny=2048, tile=32, energy_rate=0.05)
    else:
        w = wl.branched_world(0, 2048, 2048, 26500)
        p = sim.Params(nx=2048, ny=2048, tile=32)
    print(f"{case}: {w.n_particles} nodes, {w.n_filaments} filaments", flush=True)
    W = sim.World(w, p)
    W.rollout(0, n)
    W.sync()
    op = oracle_params(p)
    ex, ea, eu, ed = final_state_errors(w, W.state, op, 0, n)
    print(f"{case}, {n} steps: e_x={ex:.2e} e_a={ea:.2e} cells e_u={eu:.2e} e_d={ed:.2e}")
    assert ex <= TOL_X and eu <= TOL_U and ed <= TOL_D
    if case.startswith("energy"):
        inp = O.inputs_from_world(w)
        x, f = O.positions_from_world(w), O.rest_populations(op)
        E = torch.tensor(w.energy, dtype=DT)
        topo = inp.topo
        collected = torch.zeros(w.n_filaments, dtype=DT)
        with torch.no_grad():
            for t in range(n):
                e, col, E = O.energy_update(x, E, topo, p.energy_rate, op)
                collected += col
                x, f, _ = O.step(x, f, t, inp, op)
        errs = [rel(W.state.energy.cpu().double().numpy(), E.numpy()),
                rel(W.state.energy_sensed.cpu().double().numpy(), e.numpy()),
                rel(W.state.energy_collected.cpu().double().numpy(), collected.numpy())]
        print(f"  energy: field {errs[0]:.2e} sensed {errs[1]:.2e} collected {errs[2]:.2e}")
        assert max(errs) <= TOL_E
    W.close()
