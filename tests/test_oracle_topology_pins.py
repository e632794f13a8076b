"""Pins of the oracle's filament generality (Methods, Filaments: per-edge
stiffness coefficients; loops with a graph representation; Experiments, QD
Search, Eqs. 5-6: bending and stretching effort).

  * colouring: in every Gauss-Seidel colour no two edges share a node and no
    two joints share an edge; each edge and joint is in exactly one colour;
    loops of odd length need the third colour, even ones do not (brute force);
  * a regular polygon loop at its rest shape (unit sides, rest angles 2 pi/n)
    feels no elastic force, for odd and even n; a perturbed loop's elastic
    forces sum to zero and rotate with it;
  * per-edge stiffness: arrays equal to the scalars change nothing; with the
    first edge's stretch stiffness 0, the first node is never moved (no other
    edge touches it); with every bending stiffness 0 the edge angles leave
    the bending pass unchanged;
  * efforts: the closed form of one change, end nodes of a chain excluded,
    every node of a loop included.
Each is run against a planted mistake (the closing edge dropped from a loop,
stiffness read one edge off), which it must reject.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O

DT = torch.float64


def _polygon(n, centre=(20.0, 20.0)):
    r = 0.5 / math.sin(math.pi / n)                   # unit sides
    a = 2 * math.pi * np.arange(n) / n
    return torch.tensor(np.stack([centre[0] + r * np.cos(a), centre[1] + r * np.sin(a)]), dtype=DT)


@pytest.mark.parametrize("n", [3, 4, 7, 10, 11])
def test_colouring_of_chains_and_loops(n):
    topo = O.Topology(np.array([0, n, n + 5, 2 * n + 5]), closed=[True, False, True])
    seen_e, seen_j = [], []
    for es in topo.edge_sets:
        nodes = torch.cat([es, topo.edge_next[es]]).tolist()
        assert len(nodes) == len(set(nodes))
        seen_e += es.tolist()
    for js in topo.joint_sets:
        used = torch.cat([js, topo.joint_prev[js]]).tolist()      # the two edges of each joint
        assert len(used) == len(set(used))
        seen_j += js.tolist()
    assert sorted(seen_e) == sorted(topo.edges.tolist()) and len(seen_e) == len(set(seen_e))
    assert sorted(seen_j) == sorted(topo.joints.tolist()) and len(seen_j) == len(set(seen_j))
    assert len(topo.edges) == n + 4 + n and len(topo.joints) == n + 3 + n
    assert (topo.edge_sets[2].numel() > 0) == (n % 2 == 1)


@pytest.mark.parametrize("n", [5, 8, 13])
def test_polygon_loop_at_rest_feels_no_force(n):
    x = _polygon(n)
    topo = O.Topology(np.array([0, n]), closed=[True])
    th = torch.full((n,), 2 * math.pi / n, dtype=DT)
    L = torch.ones(n, dtype=DT)
    F = O.elastic_force(x, topo, th, L, O.Params(nx=64, ny=64))
    assert float(F.abs().max()) < 1e-12
    # the same ring without its closing edge is a chain: the end nodes are
    # no longer held and the rest angles at the ends do not apply, so a
    # bent chain with the loop's angles still sits at rest ...
    chain = O.Topology(np.array([0, n]))
    Fc = O.elastic_force(x, chain, th, L, O.Params(nx=64, ny=64))
    assert float(Fc.abs().max()) < 1e-12
    # ... but a stretched closing edge is felt only by the loop
    xs = x.clone()
    xs[:, 0] += torch.tensor([-0.3, 0.1], dtype=DT)
    Fl = O.elastic_force(xs, topo, th, L, O.Params(nx=64, ny=64))
    Fo = O.elastic_force(xs, chain, th, L, O.Params(nx=64, ny=64))
    assert float((Fl - Fo).abs().max()) > 1e-3


def test_perturbed_loop_forces_sum_to_zero_and_rotate():
    n = 9
    rng = np.random.default_rng(2)
    x = _polygon(n) + torch.tensor(rng.normal(0, 0.15, size=(2, n)), dtype=DT)
    topo = O.Topology(np.array([0, n]), closed=[True])
    th = torch.tensor(2 * math.pi / n + rng.normal(0, 0.2, size=n), dtype=DT)
    L = torch.tensor(1 + rng.normal(0, 0.1, size=n), dtype=DT)
    p = O.Params(nx=64, ny=64)
    F = O.elastic_force(x, topo, th, L, p)
    assert float(F.sum(dim=1).abs().max()) < 1e-13
    c, s = math.cos(0.7), math.sin(0.7)
    R = torch.tensor([[c, -s], [s, c]], dtype=DT)
    Fr = O.elastic_force(R @ x, topo, th, L, p)
    assert float((Fr - R @ F).abs().max()) < 1e-12


def _chain_case():
    x = torch.tensor([[0.0, 1.3, 2.1, 3.4, 4.0], [0.0, 0.4, 1.5, 1.2, 2.0]], dtype=DT)
    topo = O.Topology(np.array([0, 5]))
    th = torch.tensor([0.0, 0.35, -0.6, 0.2, 0.0], dtype=DT)
    L = torch.tensor([1.1, 0.9, 1.25, 1.0, 0.0], dtype=DT)
    return x, topo, th, L, O.Params(nx=64, ny=64, k_bend=0.7, k_stretch=0.9, k_shear=0.4)


def pin_first_edge_free(project):
    x, topo, th, L, p = _chain_case()
    kb = torch.full((5,), 0.7, dtype=DT)
    ks = torch.full((5,), 0.9, dtype=DT)
    ksh = torch.full((5,), 0.4, dtype=DT)
    y_arr, _ = project(x, topo, th, L, p, (kb, ks, ksh))
    y_sc, _ = O.pbd_project(x, topo, th, L, p)
    assert float((y_arr - y_sc).abs().max()) < 1e-15        # arrays equal to the scalars
    ks0 = ks.clone()
    ks0[0] = 0.0
    y, _ = project(x, topo, th, L, p, (kb, ks0, ksh))
    assert float((y[:, 0] - x[:, 0]).abs().max()) == 0.0     # node 0 only has edge 0
    assert float((y[:, 1] - x[:, 1]).abs().max()) > 1e-3     # edge 1 still moves node 1


def test_per_edge_stiffness_pins():
    pin_first_edge_free(lambda x, topo, th, L, p, st: O.pbd_project(x, topo, th, L, p, stiff=st))
    # no bending stiffness anywhere: the bending pass leaves the angles alone
    x, topo, th, L, p = _chain_case()
    zero = torch.zeros(5, dtype=DT)
    _, theta = O.pbd_project(x, topo, th, L, p, iters=1,
                             stiff=(zero, torch.zeros(5, dtype=DT), torch.zeros(5, dtype=DT)))
    assert float((theta - O.edge_angles(x, topo)).abs().max()) == 0.0


def test_planted_mistake_stiffness_off_by_one_edge():
    def shifted(x, topo, th, L, p, st):
        kb, ks, ksh = st
        return O.pbd_project(x, topo, th, L, p, stiff=(kb, torch.roll(ks, 1), ksh))
    with pytest.raises(AssertionError):
        pin_first_edge_free(shifted)


def test_planted_mistake_loop_without_closing_edge():
    n = 8
    x = _polygon(n)
    x[:, 0] += torch.tensor([-0.3, 0.1], dtype=DT)
    th = torch.full((n,), 2 * math.pi / n, dtype=DT)
    L = torch.ones(n, dtype=DT)
    loop = O.Topology(np.array([0, n]), closed=[True])
    F = O.elastic_force(x, loop, th, L, O.Params(nx=64, ny=64))
    broken = O.Topology(np.array([0, n]), closed=[True])
    keep = broken.edges != n - 1
    broken.edges = broken.edges[keep]
    broken.edge_sets = [es[es != n - 1] for es in broken.edge_sets]
    Fb = O.elastic_force(x, broken, th, L, O.Params(nx=64, ny=64))
    assert float((F - Fb).abs().max()) > 1e-3


def test_effort_closed_form():
    topo = O.Topology(np.array([0, 5, 9]), closed=[False, True])
    old_a = torch.zeros(9, dtype=DT)
    new_a = torch.arange(9, dtype=DT) * 0.1
    old_l = torch.ones(9, dtype=DT)
    new_l = 1 + torch.arange(9, dtype=DT) * 0.01
    E = O.rest_effort(topo, old_a, new_a, old_l, new_l)
    # chain 0..4: joints 1, 2, 3; edges 0..3.  loop 5..8: joints and edges 5..8
    want_b = [sum((0.1 * i) ** 2 for i in (1, 2, 3)), sum((0.1 * i) ** 2 for i in (5, 6, 7, 8))]
    want_p = [sum((0.01 * i) ** 2 for i in (0, 1, 2, 3)), sum((0.01 * i) ** 2 for i in (5, 6, 7, 8))]
    assert np.allclose(E[0].numpy(), want_b, rtol=1e-14) and np.allclose(E[1].numpy(), want_p, rtol=1e-14)
    # a change at a chain's end node is no joint: no bending effort
    bump = old_a.clone()
    bump[0] = 1.0
    bump[4] = 1.0
    assert float(O.rest_effort(topo, old_a, bump, old_l, old_l)[0, 0]) == 0.0


def test_loop_actuation_wave_uses_all_joints():
    n = 8
    topo = O.Topology(np.array([0, n]), closed=[True])
    ra = torch.zeros(n, dtype=DT)
    amp, period, phase = torch.tensor([0.5], dtype=DT), torch.tensor([40.0], dtype=DT), torch.tensor([0.0], dtype=DT)
    th = O.actuation(ra, topo, amp, period, phase, 10)       # 2 pi t / T = pi / 2
    want = 0.5 * np.sin(np.pi / 2 - 2 * np.pi * np.arange(n) / n)
    assert np.allclose(th.numpy(), want, atol=1e-15)
