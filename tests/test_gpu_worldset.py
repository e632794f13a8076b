"""A set of worlds stepped and differentiated together in the same launches
(sim_create_set): each world's trajectory and gradients equal the same world
run alone (bit for bit: the binned transfer's sums are fixed point and every
kernel reads its world's own buffers), and one world's gradient matches the
FP64 oracle's reverse mode (normwise relative <= 1e-3, cosine >= 0.9999);
with multi-direct forcing and with two-layer markers as well; the
single-world test hooks refuse sets.
"""
import numpy as np
import pytest
import torch

from paper_2607_02954_amd import workloads as wl
from test_gpu_adjoint import _compare, _joints, _oracle_grad

pytestmark = pytest.mark.gpu


def _sim():
    from paper_2607_02954_amd import sim
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sim


def _worlds():
    return [wl.random_world(21, 80, 64, [12, 30, 7], amp=0.5), wl.random_world(22, 80, 64, [40, 2], amp=0.5),
            wl.random_world(23, 80, 64, [9, 9, 9, 20], amp=0.5)]


def _targets(worlds):
    g = np.random.default_rng(4)
    return [w.positions64() + g.normal(0, 0.5, size=(2, w.n_particles)) for w in worlds]


def _loss(x, tgts, n_parts):
    off, loss = 0, 0.0
    for t, n in zip(tgts, n_parts):
        xw = x[off:off + 2 * n].reshape(2, n)
        loss = loss + ((xw - t) ** 2).sum() / n
        off += 2 * n
    return loss


@pytest.mark.parametrize("mdf,offset", [(1, 0.0), (3, 0.0), (3, 0.5)])
def test_set_equals_worlds_alone_and_the_oracle(mdf, offset):
    sim = _sim()
    worlds = _worlds()
    p = sim.Params(nx=80, ny=64, mdf_iters=mdf, marker_offset=offset)
    n, k = 14, 5
    S = sim.WorldSet(worlds, p)
    tg = [torch.tensor(t, dtype=torch.float64, device="cuda") for t in _targets(worlds)]
    ra = torch.tensor(np.concatenate([w.rest_angle for w in worlds]), dtype=torch.float64, device="cuda",
                      requires_grad=True)
    x = sim.SetRollout.apply(ra, S, 0, n, k)
    _loss(x, tg, S.n_parts).backward()
    torch.cuda.synchronize()
    g_set = ra.grad.cpu().numpy()
    off = 0
    for i, w in enumerate(worlds):
        W = sim.World(w, p)
        raw = torch.tensor(w.rest_angle, dtype=torch.float64, device="cuda", requires_grad=True)
        xw = sim.Rollout.apply(raw, W, 0, n, k)
        (((xw - tg[i]) ** 2).sum() / w.n_particles).backward()
        torch.cuda.synchronize()
        for key in ("cell", "frac", "f", "u"):
            assert torch.equal(getattr(S.states[i], key), getattr(W.state, key)), (i, key)
        g_one = raw.grad.cpu().numpy()
        d = float(np.abs(g_set[off:off + w.n_particles] - g_one).max())
        print(f"MDF {mdf}, offset {offset}, world {i} (N={w.n_particles}): set vs alone max |dg| = {d:.1e}")
        assert np.array_equal(g_set[off:off + w.n_particles], g_one)
        if i == 1:
            ref, _ = _oracle_grad(w, p, _targets(worlds)[i], n, k)
            err, cos = _compare(g_one, ref, _joints(w))
            print(f"  vs oracle: rel err {err:.2e} cos {cos:.6f}")
            assert err <= 1e-3 and cos >= 0.9999
        off += w.n_particles


def test_set_refuses_single_world_hooks():
    sim = _sim()
    S = sim.WorldSet(_worlds(), sim.Params(nx=80, ny=64))
    for call in (lambda: sim.check(sim.lib().sim_debug_substep(S.handle, 0, 0)),
                 lambda: sim.check(sim.lib().sim_profile_steps(S.handle, 0, 1, (sim.ctypes.c_float * 6)()))):
        with pytest.raises(sim.SimError) as ei:
            call()
        assert ei.value.status == sim.SIM_E_INVALID
