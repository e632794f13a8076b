"""Closed-form pins of the oracle's PBD pass order and actuation law.

Methods, Filaments: one PBD iteration is first a bending pass (Eq. 1) over the
joints, then a position pass (Eqs. 2-4) over the edges; the reading used here
sweeps each pass in two colours, even local index first, and applies every
constraint to the current values (Gauss-Seidel).  With unit stiffnesses, one
iteration on a four-node chain has closed-form consequences that hold only
for that order:
  * the odd joint (the last bending update) is solved exactly:
    theta_2 - theta_1 = theta_hat at the third node;
  * edge 0 is touched only by the even joint, once, from the initial angles:
    theta_0' = theta_0 + (wrap(theta_1 - theta_0) - theta_hat) / 2;
  * the odd edge (the last position update) ends exactly on its rest shape:
    y_2 - y_1 = L_1 d(theta_1'), with the angles after the bending pass;
  * the end nodes are touched only by their even edges, once, from the
    initial positions: y_0' = y_0 + (v_0 - L_0 d(theta_0')) / 2, and the
    mirror image at node 3;
  * the angle sum and the centroid are unchanged (Eqs. 1 and 4).
Experiments, Hand-designed locomotion (sinusoidal wave, one wavelength per
body): the actuated rest angle theta_rest + A sin(2 pi t / T + psi -
2 pi k / (n - 2)) is pinned at points where the sine is exactly 0 or +-1.

Each pin is also run against planted mistakes (the oracle's own building
blocks composed in a wrong order, or a wrong actuation formula), which it
must reject.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O

DT = torch.float64


# ----------------------------------------------------------------------------
# PBD pass order
# ----------------------------------------------------------------------------

def _chain4():
    # a bent, stretched four-node chain: every constraint is active
    x = torch.tensor([[0.0, 1.3, 2.1, 3.4], [0.0, 0.4, 1.5, 1.2]], dtype=DT)
    topo = O.Topology(np.array([0, 4]))
    theta_hat = torch.tensor([0.0, 0.35, -0.6, 0.0], dtype=DT)
    L = torch.tensor([1.1, 0.9, 1.25, 0.0], dtype=DT)
    p = O.Params(nx=64, ny=64, k_bend=1.0, k_stretch=1.0, k_shear=1.0, pbd_iters=1)
    return x, topo, theta_hat, L, p


def _d(th):
    return torch.stack([torch.cos(th), torch.sin(th)])


def _pins(x, topo, theta_hat, L, y, th):
    """Closed-form consequences of one ordered iteration with unit stiffnesses;
    returns the largest violation."""
    th0 = O.edge_angles(x, topo)
    v = x[:, 1:] - x[:, :-1]
    errs = [
        abs(float(O.wrap_angle(th[2] - th[1]) - theta_hat[2])),
        abs(float(th[0] - (th0[0] + 0.5 * (O.wrap_angle(th0[1] - th0[0]) - theta_hat[1])))),
        abs(float(th[:3].sum() - th0[:3].sum())),
        float(torch.max(torch.abs((y[:, 2] - y[:, 1]) - L[1] * _d(th[1])))),
        float(torch.max(torch.abs(y[:, 0] - (x[:, 0] + 0.5 * (v[:, 0] - L[0] * _d(th[0])))))),
        float(torch.max(torch.abs(y[:, 3] - (x[:, 3] - 0.5 * (v[:, 2] - L[2] * _d(th[2])))))),
        float(torch.max(torch.abs(y.sum(dim=1) - x.sum(dim=1)))),
    ]
    return max(errs)


def _variant(kind, x, topo, theta_hat, L, p):
    """One iteration composed from the oracle's passes in a wrong order."""
    th = O.edge_angles(x, topo)
    y = x
    jsets, esets = list(topo.joint_sets), list(topo.edge_sets)
    if kind in ("odd_first", "bend_odd_first"):
        jsets = jsets[::-1]
    if kind in ("odd_first", "pos_odd_first"):
        esets = esets[::-1]

    def bend(th):
        if kind == "jacobi":
            j = topo.joints
            c = O.wrap_angle(th[j] - th[j - 1]) - theta_hat[j]
            return th.index_add(0, j - 1, 0.5 * p.k_bend * c).index_add(0, j, -0.5 * p.k_bend * c)
        for js in jsets:
            th = O.bend_pass(th, js, theta_hat, p.k_bend)
        return th

    def position(y, th):
        if kind == "jacobi":
            return O.position_pass(y, th, topo.edges, L, p.k_stretch, p.k_shear)
        for es in esets:
            y = O.position_pass(y, th, es, L, p.k_stretch, p.k_shear)
        return y

    if kind == "position_first":
        y = position(y, th)
        th = bend(th)
    else:
        th = bend(th)
        y = position(y, th)
    return y, th


def test_one_iteration_closed_forms_hold():
    x, topo, theta_hat, L, p = _chain4()
    y, th = O.pbd_project(x, topo, theta_hat, L, p)
    assert _pins(x, topo, theta_hat, L, y, th) < 1e-14
    # the force is k_el times the projection's displacement (node 0 closed form)
    F = O.elastic_force(x, topo, theta_hat, L, p)
    v0 = x[:, 1] - x[:, 0]
    assert torch.max(torch.abs(F[:, 0] - p.k_elastic * 0.5 * (v0 - L[0] * _d(th[0])))) < 1e-15


@pytest.mark.parametrize("kind", ["position_first", "odd_first", "bend_odd_first", "pos_odd_first", "jacobi"])
def test_closed_forms_reject_planted_order_mistakes(kind):
    x, topo, theta_hat, L, p = _chain4()
    y, th = _variant(kind, x, topo, theta_hat, L, p)
    assert _pins(x, topo, theta_hat, L, y, th) > 1e-3, kind


def test_variant_harness_reproduces_the_oracle_order():
    # the harness composed in the right order is the oracle itself
    x, topo, theta_hat, L, p = _chain4()
    y, th = _variant("ordered", x, topo, theta_hat, L, p)
    y0, th0 = O.pbd_project(x, topo, theta_hat, L, p)
    assert torch.equal(y, y0) and torch.equal(th, th0)


# ----------------------------------------------------------------------------
# Actuation law
# ----------------------------------------------------------------------------

# n = 6 nodes: joints at nodes 1..4, local index k = 0..3, n - 2 = 4
_REST = torch.tensor([0.0, 0.11, -0.23, 0.31, 0.05, 0.0], dtype=DT)
_JOINT = [1, 2, 3, 4]
A, T = 0.5, 40.0
# (t, psi) -> expected actuation offset of joints k = 0..3
_CASES = [
    (10.0, 0.0, [A, 0.0, -A, 0.0]),                  # t = T/4: sin(pi/2 - pi k/2)
    (0.0, math.pi / 2, [A, 0.0, -A, 0.0]),           # the phase alone: sin(pi/2 - pi k/2)
    (0.0, 0.0, [0.0, -A, 0.0, A]),                   # travelling term: sin(-pi k/2)
    (30.0, math.pi, [A, 0.0, -A, 0.0]),              # sin(3 pi/2 + pi - pi k/2)
]


def _act_errors(fn):
    topo = O.Topology(np.array([0, 6]))
    amp, period = torch.tensor([A], dtype=DT), torch.tensor([T], dtype=DT)
    worst = 0.0
    for t, psi, expect in _CASES:
        got = fn(_REST, topo, amp, period, torch.tensor([psi], dtype=DT), t)
        for j, e in zip(_JOINT, expect):
            worst = max(worst, abs(float(got[j]) - (float(_REST[j]) + e)))
        worst = max(worst, abs(float(got[0] - _REST[0])), abs(float(got[5] - _REST[5])))
    return worst


def test_actuation_closed_form_values():
    assert _act_errors(O.actuation) < 1e-15


def _planted(kind):
    def fn(rest, topo, amp, period, phase, t):
        f = topo.joint_fil
        k = topo.joint_local.to(DT)
        n2 = topo.joint_count.to(DT)
        if kind == "cos":
            off = amp[f] * torch.cos(2 * math.pi * t / period[f] + phase[f] - 2 * math.pi * k / n2)
        elif kind == "no_phase":
            off = amp[f] * torch.sin(2 * math.pi * t / period[f] - 2 * math.pi * k / n2)
        elif kind == "wave_sign":
            off = amp[f] * torch.sin(2 * math.pi * t / period[f] + phase[f] + 2 * math.pi * k / n2)
        elif kind == "n_minus_1":
            off = amp[f] * torch.sin(2 * math.pi * t / period[f] + phase[f] - 2 * math.pi * k / (n2 + 1))
        else:                                            # "no_two_pi_t"
            off = amp[f] * torch.sin(t / period[f] + phase[f] - 2 * math.pi * k / n2)
        return rest.clone().index_add(0, topo.joints, off)
    return fn


@pytest.mark.parametrize("kind", ["cos", "no_phase", "wave_sign", "n_minus_1", "no_two_pi_t"])
def test_actuation_pins_reject_planted_mistakes(kind):
    assert _act_errors(_planted(kind)) > 1e-2, kind
