"""Pins of the oracle's filament generality (Methods, Filaments: per-edge
stiffness coefficients; loops and branches with a graph representation;
Discussion: cactus graphs; Experiments, QD
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
  * branches (a filament hanging from a node of an earlier one): a branch at
    the second node of a two-node parent gives the chain through the same
    nodes to the last bit (its Gauss-Seidel order agrees with the chain's on
    every pair of constraints that share a variable); a T-junction at its
    rest shape feels no force; a branched creature's forces sum to zero and
    rotate with it; topologies that are not cactus trees of chains and loops
    are refused.
Each is run against a planted mistake (the closing edge dropped from a loop,
stiffness read one edge off, the attachment's rest angles swapped, its
joints before the regular colours or with the wrong sign, its edge
dropped), which it must reject.
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


# ---------------------------------------------------------------------------
# Branches: a filament hanging from a node of an earlier one
# ---------------------------------------------------------------------------

def _params(**kw):
    return O.Params(nx=64, ny=64, **kw)


def _branch_pair(m, L0=1.1, La=0.9, alpha=0.4, beta=-0.3, seed=0):
    """A 2-node parent with an m-node child at its second node, and the
    (m + 2)-node chain through the same nodes: its joints at the parent's
    second node and the child's first carry alpha and beta, its edge between
    them the attachment's rest length."""
    g = np.random.default_rng(seed)
    n = m + 2
    ang = np.cumsum(g.normal(0.0, 0.35, size=n - 1))
    x = np.zeros((2, n))
    x[:, 0] = (30.0, 30.0)
    for i in range(1, n):
        x[:, i] = x[:, i - 1] + (1.0 + 0.1 * g.normal()) * np.array([math.cos(ang[i - 1]), math.sin(ang[i - 1])])
    x = torch.tensor(x, dtype=DT)
    rl = torch.tensor(1.0 + 0.2 * g.uniform(size=n), dtype=DT)
    ra = torch.tensor(g.normal(0.0, 0.3, size=n), dtype=DT)
    # the chain
    chain = O.Topology(np.array([0, n]))
    rl_c, ra_c = rl.clone(), ra.clone()
    rl_c[0], rl_c[1] = L0, La
    ra_c[1], ra_c[2] = alpha, beta
    # the branch: filament 0 = nodes 0, 1; filament 1 = nodes 2 .. n-1 hanging from node 1
    att = np.zeros((3, 2))
    att[:, 1] = (La, alpha, beta)
    branch = O.Topology(np.array([0, 2, n]), parent=[-1, 1], attach=att)
    rl_b, ra_b = rl.clone(), ra.clone()
    rl_b[0] = L0
    return x, (chain, ra_c, rl_c), (branch, ra_b, rl_b)


@pytest.mark.parametrize("m", [1, 2, 3, 6])
def test_branch_at_a_two_node_parent_is_the_chain(m):
    """The Gauss-Seidel order of the branch (regular colours, then the joint
    at the parent node, then the one at the child's first node; regular
    edges, then the attachment edge) orders every pair of constraints that
    share a variable as the chain's two colours do, so the projections agree
    to the last bit."""
    x, (chain, ra_c, rl_c), (branch, ra_b, rl_b) = _branch_pair(m)
    p = _params()
    y_c, th_c = O.pbd_project(x, chain, ra_c, rl_c, p)
    y_b, th_b = O.pbd_project(x, branch, ra_b, rl_b, p)
    assert torch.equal(y_b, y_c)
    # the child's edge angles are the chain's (the attachment edge has no node slot in the branch)
    assert torch.equal(th_b[2:n_edges(m)], th_c[2:n_edges(m)])


def n_edges(m):
    return m + 1


def test_t_junction_at_rest_feels_no_force():
    """A straight 5-node parent along x with a 3-node child leaving its middle
    node straight up (attachment rest length 1, angle +pi/2 from the parent's
    entering edge, 0 at the child) is at rest."""
    x = torch.tensor([[10.0, 11, 12, 13, 14, 12, 12, 12], [20.0, 20, 20, 20, 20, 21, 22, 23]], dtype=DT)
    topo = O.Topology(np.array([0, 5, 8]), parent=[-1, 2], attach=np.array([[0.0, 1.0], [0.0, math.pi / 2], [0.0, 0.0]]))
    ra = torch.zeros(8, dtype=DT)
    rl = torch.ones(8, dtype=DT)
    F = O.elastic_force(x, topo, ra, rl, _params())
    assert float(F.abs().max()) <= 1e-14
    # planted mistake: the two rest angles of the attachment swapped
    swapped = O.Topology(np.array([0, 5, 8]), parent=[-1, 2], attach=np.array([[0.0, 1.0], [0.0, 0.0], [0.0, math.pi / 2]]))
    assert float(O.elastic_force(x, swapped, ra, rl, _params()).abs().max()) > 1e-3


def _creature(seed=3):
    """A loop with a chain hanging from one of its nodes and a grandchild on
    the chain."""
    g = np.random.default_rng(seed)
    loop = _polygon(6, centre=(13.0, 21.5)).numpy()
    chain = np.stack([14.0 + np.arange(8), np.full(8, 20.0)])
    kid = np.stack([16.0 + np.arange(4), np.full(4, 24.0)])
    x = torch.tensor(np.concatenate([loop, chain, kid], axis=1) + 0.15 * g.normal(size=(2, 18)), dtype=DT)
    att = np.zeros((3, 3))
    att[:, 1] = (1.2, 1.0, 0.2)
    att[:, 2] = (0.8, -0.7, 0.3)
    with pytest.raises(ValueError):                      # a closed loop cannot hang from a node
        O.Topology(np.array([0, 6, 14, 18]), closed=[True, True, False], parent=[-1, 0, 10], attach=att)
    topo = O.Topology(np.array([0, 6, 14, 18]), closed=[True, False, False], parent=[-1, 0, 10], attach=att)
    ra = torch.tensor(g.normal(0, 0.3, size=18), dtype=DT)
    rl = torch.tensor(1.0 + 0.1 * g.uniform(size=18), dtype=DT)
    return x, topo, ra, rl


def test_branched_forces_sum_to_zero_and_rotate():
    x, topo, ra, rl = _creature()
    p = _params()
    F = O.elastic_force(x, topo, ra, rl, p)
    assert float(F.abs().max()) > 1e-4
    assert float(F.sum(dim=1).abs().max()) <= 1e-15
    c, s = math.cos(0.7), math.sin(0.7)
    R = torch.tensor([[c, -s], [s, c]], dtype=DT)
    F_rot = O.elastic_force(R @ x + 5.0, topo, ra, rl, p)
    assert float((F_rot - R @ F).abs().max()) <= 1e-12


def test_branch_topologies_that_are_not_cactus_trees_are_refused():
    att = np.ones((3, 3))
    with pytest.raises(ValueError):                      # parent node in a later filament
        O.Topology(np.array([0, 4, 8, 12]), parent=[5, -1, -1], attach=att)
    with pytest.raises(ValueError):                      # two filaments on one node
        O.Topology(np.array([0, 4, 8, 12]), parent=[-1, 2, 2], attach=att)
    with pytest.raises(ValueError):                      # parent node without an entering edge
        O.Topology(np.array([0, 4, 8, 12]), parent=[-1, 0, -1], attach=att)
    O.Topology(np.array([0, 4, 8, 12]), closed=[True, False, False], parent=[-1, 0, 5], attach=att)   # a loop's first node has one


def _project_variant(x, topo, theta_hat, rest_length, p, variant):
    """pbd_project with one planted mistake."""
    y = x
    theta = O.edge_angles(y, topo)
    th_att = O.attachment_angles(y, topo)
    for _ in range(p.pbd_iters):
        if variant == "attachments first":
            theta, th_att = O.bend_attachments(theta, th_att, topo, p.k_bend)
        for js in topo.joint_sets:
            theta = O.bend_pass(theta, js, theta_hat, p.k_bend, topo.joint_prev)
        if variant == "sign":
            theta, th_att = O.bend_attachments(theta, th_att, topo, -p.k_bend)
        elif variant != "attachments first":
            theta, th_att = O.bend_attachments(theta, th_att, topo, p.k_bend)
        for es in topo.edge_sets:
            y = O.position_pass(y, theta, es, rest_length, p.k_stretch, p.k_shear, topo.edge_next)
        if variant != "no attachment edge":
            y = O.position_attachments(y, th_att, topo, p.k_stretch, p.k_shear)
    return y


@pytest.mark.parametrize("variant", ["attachments first", "sign", "no attachment edge"])
def test_planted_mistakes_in_the_branch_break_the_chain_pin(variant):
    x, (chain, ra_c, rl_c), (branch, ra_b, rl_b) = _branch_pair(5)
    p = _params()
    y_c, _ = O.pbd_project(x, chain, ra_c, rl_c, p)
    y_ok = _project_variant(x, branch, ra_b, rl_b, p, "none")
    assert torch.equal(y_ok, y_c)
    y_bad = _project_variant(x, branch, ra_b, rl_b, p, variant)
    assert float((y_bad - y_c).abs().max()) > 1e-6
