"""Pins of the oracle's energy field (Methods, Fields; Experiments,
Neuroevolution of Controller Circuit: energy packets, sensing at the node,
energy collected).

  * a packet's peak is its amplitude at its centre; a cell one width away
    holds A e^{-1/2}; the field is periodic (a packet moved by the period is
    the same field);
  * mass balance: the field loses exactly what the nodes collect, step after
    step, and the filaments' collected totals add up to it;
  * a single node resting on a cell centre in a uniform field senses the
    field value and, step after step, its sensed value decays geometrically
    by 1 - rate (3/8)^2, (3/8 being the sum of the squared 1D weights of the
    4-point function at a cell centre: 1/16 + 1/4 + 1/16);
  * rate 0 changes nothing.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O

DT = torch.float64


def test_packet_values_and_periodicity():
    nx, ny = 40, 30
    c = torch.tensor([[10.0], [7.0]], dtype=DT)
    E = O.energy_packets(nx, ny, c, torch.tensor([2.5], dtype=DT), torch.tensor([3.0], dtype=DT))
    assert abs(float(E[7, 10]) - 2.5) < 1e-15
    assert abs(float(E[7, 13]) - 2.5 * math.exp(-0.5)) < 1e-14
    assert abs(float(E[10, 10]) - 2.5 * math.exp(-0.5)) < 1e-14
    E2 = O.energy_packets(nx, ny, c + torch.tensor([[nx], [-ny]], dtype=DT), torch.tensor([2.5], dtype=DT),
                          torch.tensor([3.0], dtype=DT))
    assert float((E - E2).abs().max()) < 1e-12


def test_mass_balance_over_steps():
    nx, ny = 48, 40
    rng = np.random.default_rng(1)
    E = O.energy_packets(nx, ny, torch.tensor(rng.uniform(0, 40, size=(2, 5)), dtype=DT),
                         torch.tensor(rng.uniform(0.5, 2, size=5), dtype=DT),
                         torch.tensor(rng.uniform(2, 6, size=5), dtype=DT))
    topo = O.Topology(np.array([0, 7, 9, 20]))
    p = O.Params(nx=nx, ny=ny)
    x = torch.tensor(rng.uniform(0, 40, size=(2, 20)), dtype=DT)
    total = torch.zeros(3, dtype=DT)
    E0 = float(E.sum())
    for _ in range(5):
        before = float(E.sum())
        e, coll, E = O.energy_update(x, E, topo, 0.2, p)
        assert abs(before - float(E.sum()) - float(coll.sum())) < 1e-12
        assert abs(float(coll.sum()) - 0.2 * float(e.sum())) < 1e-12
        total = total + coll
        x = x + 0.3
    assert abs(E0 - float(E.sum()) - float(total.sum())) < 1e-11


def test_single_node_geometric_decay():
    nx = ny = 16
    p = O.Params(nx=nx, ny=ny)
    E = torch.full((ny, nx), 3.0, dtype=DT)
    topo = O.Topology(np.array([0, 1]))
    x = torch.tensor([[5.0], [9.0]], dtype=DT)
    rate = 0.4
    ratio = 1 - rate * (3 / 8) ** 2
    e, _, E = O.energy_update(x, E, topo, rate, p)
    assert abs(float(e[0]) - 3.0) < 1e-14
    for k in range(1, 6):
        e, _, E = O.energy_update(x, E, topo, rate, p)
        assert abs(float(e[0]) - 3.0 * ratio ** k) < 1e-13, k
    E1 = torch.full((ny, nx), 3.0, dtype=DT)
    _, coll, E2 = O.energy_update(x, E1, topo, 0.0, p)
    assert float(coll.abs().max()) == 0.0 and torch.equal(E1, E2)


def _update_mistake(kind):
    def fn(x, E, topo, rate, p):
        e = O.interpolate(x, E[None], p)[0]
        c = rate * e
        coll = torch.zeros(topo.n_filaments, dtype=DT).index_add(0, topo.fil_of_node, c)
        if kind == "no depletion":
            return e, coll, E
        # taken out of the nearest cell only
        E = E.clone()
        ix = torch.remainder(torch.round(x[0]).long(), p.nx)
        iy = torch.remainder(torch.round(x[1]).long(), p.ny)
        E.index_put_((iy, ix), -c, accumulate=True)
        return e, coll, E
    return fn


@pytest.mark.parametrize("kind", ["no depletion", "nearest cell"])
def test_planted_mistakes_are_caught(kind, monkeypatch):
    monkeypatch.setattr(O, "energy_update", _update_mistake(kind))
    with pytest.raises(AssertionError):
        test_mass_balance_over_steps()
        test_single_node_geometric_decay()
