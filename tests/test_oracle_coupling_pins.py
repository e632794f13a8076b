"""Pins of the oracle's leakage fixes (Methods, Fluid-filament Interaction:
Multi-Direct Forcing; the filament broadcast as a two-layer version of
itself).

  * markers: a straight chain along x has normals (0, 1) at every node; a
    regular polygon loop has unit normals along the radius;
  * the two-layer spread conserves what is spread (sum over cells = sum over
    nodes), and as delta -> 0 it tends to the one-layer spread as delta^2
    (the two markers are symmetric about the node);
  * MDF on a single node at a cell centre in fluid at rest: with
    a = sum_c W^2 = (3/8)^2 the k-th correction starts from a mismatch of
    (F/2) (1 - a)^(k-1) (closed form of the fixed-point iteration);
  * MDF iterations drive the marker velocity of nodes far apart to the
    desired velocity (no slip at the markers) geometrically, at least 10% per
    iteration; on unit-spaced
    chains (a strongly coupled, ill-conditioned system) the mismatch still
    falls monotonically.
  * the reverse mode through the two-layer transfers (the markers' normals
    as functions of the neighbouring nodes included) agrees with central
    differences, and stays finite where a single-node filament has no
    normal (its markers sit on the node; the derivative there is zero).
Planted mistakes (markers both on one side, the correction without its
factor 2) are rejected.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O

DT = torch.float64


def test_marker_normals():
    topo = O.Topology(np.array([0, 6]))
    x = torch.tensor([[3.0 + k for k in range(6)], [5.5] * 6], dtype=DT)
    n = O.marker_normals(x, topo)
    assert torch.allclose(n, torch.tensor([[0.0] * 6, [1.0] * 6], dtype=DT), atol=0, rtol=0)
    m = 9
    c = np.array([20.0, 18.0])
    r = 0.5 / math.sin(math.pi / m)
    a = 2 * math.pi * np.arange(m) / m
    xl = torch.tensor(np.stack([c[0] + r * np.cos(a), c[1] + r * np.sin(a)]), dtype=DT)
    nl = O.marker_normals(xl, O.Topology(np.array([0, m]), closed=[True]))
    radial = (xl - torch.tensor(c[:, None], dtype=DT)) / r
    assert float((nl.norm(dim=0) - 1).abs().max()) < 1e-14
    assert float((nl + radial).abs().max()) < 1e-12          # counter-clockwise loop: inward


def _pair():
    x = torch.tensor([[10.3, 11.25, 12.1, 13.0], [7.6, 7.9, 8.4, 8.5]], dtype=DT)
    topo = O.Topology(np.array([0, 4]))
    vals = torch.tensor([[0.3, -0.2, 0.5, 0.1], [0.05, 0.4, -0.1, 0.2]], dtype=DT)
    return x, topo, vals


def pin_two_layer_limit(spread2):
    x, topo, vals = _pair()
    p0 = O.Params(nx=32, ny=24)
    S0 = O.spread(x, vals, p0)
    errs = []
    for d in (1e-2, 1e-3):
        S = spread2(x, vals, topo, O.Params(nx=32, ny=24, marker_offset=d))
        assert abs(float(S.sum()) - float(vals.sum())) < 1e-13
        errs.append(float((S - S0).abs().max()))
    assert errs[1] < errs[0] / 50, errs                     # second order: 100x smaller per 10x


def test_two_layer_spread_pins():
    pin_two_layer_limit(O.spread2)


def test_planted_mistake_one_sided_markers():
    def one_sided(x, vals, topo, p):
        d = p.marker_offset * O.marker_normals(x, topo)
        return 0.5 * (O.spread(x + d, vals, p) + O.spread(x + 2 * d, vals, p))
    with pytest.raises(AssertionError):
        pin_two_layer_limit(one_sided)


def pin_mdf_closed_form(coupling):
    p = O.Params(nx=16, ny=16, mdf_iters=6)
    topo = O.Topology(np.array([0, 1]))
    x = torch.tensor([[6.0], [9.0]], dtype=DT)
    F = torch.tensor([[0.02], [-0.01]], dtype=DT)
    tr = {}
    coupling(x, O.rest_populations(p), F, topo, p, tr)
    a = (3 / 8) ** 2
    want = [float((F / 2).abs().max()) * (1 - a) ** k for k in range(1, 6)]
    assert np.allclose(tr["mdf_mismatch"], want, rtol=1e-12, atol=1e-18), (tr["mdf_mismatch"], want)


def test_mdf_closed_form():
    pin_mdf_closed_form(O.coupling_force)


def test_planted_mistake_correction_without_factor_two(monkeypatch):
    def wrong(x, f, force, topo, p, trace=None):
        Fg = O.spread2(x, force, topo, p)
        cx = O.C_Q[:, 0].reshape(9, 1, 1)
        cy = O.C_Q[:, 1].reshape(9, 1, 1)
        rho = f.sum(dim=0)
        j = torch.stack([(f * cx).sum(dim=0), (f * cy).sum(dim=0)])
        U_d = O.interpolate2(x, j / rho, topo, p) + 0.5 * force
        mm = []
        for _ in range(p.mdf_iters - 1):
            U = O.interpolate2(x, (j + 0.5 * Fg) / rho, topo, p)
            mm.append(float((U_d - U).abs().max()))
            Fg = Fg + O.spread2(x, U_d - U, topo, p)
        trace["mdf_mismatch"] = mm
        return Fg
    with pytest.raises(AssertionError):
        pin_mdf_closed_form(wrong)


def test_mdf_approaches_no_slip():
    # nodes far apart (6 cells: no two nodes share a cell of support, so
    # each node's two markers form their own small system) approach no slip
    # at their markers geometrically, at least 10% per iteration
    p = O.Params(nx=48, ny=48, mdf_iters=60, marker_offset=0.5)
    topo = O.Topology(np.array([0, 2, 4, 6]))
    x = torch.tensor([[5.3, 11.3, 25.7, 25.7, 34.1, 40.1], [8.8, 8.8, 20.2, 26.2, 36.9, 36.9]], dtype=DT)
    F = torch.tensor([[0.02, -0.01, 0.005, 0.0, -0.03, 0.01], [0.01, 0.02, -0.01, 0.004, 0.0, -0.02]], dtype=DT)
    tr = {}
    O.coupling_force(x, O.rest_populations(p), F, topo, p, tr)
    mm = tr["mdf_mismatch"]
    assert all(m <= mm[0] * 0.9 ** k * (1 + 1e-9) for k, m in enumerate(mm)), mm
    assert mm[-1] < 1e-3 * mm[0]
    # chains of unit spacing couple their markers strongly (the matrix has
    # small eigenvalues): the mismatch still falls monotonically
    from paper_2607_02954_amd import workloads as wl
    w = wl.random_world(3, 40, 36, [12, 8], amp=0.5)
    inp = O.inputs_from_world(w)
    x = O.positions_from_world(w)
    f = O.rest_populations(O.Params(nx=40, ny=36))
    for t in range(3):                                      # a developed flow first
        x, f, _ = O.step(x, f, t, inp, O.Params(nx=40, ny=36))
    tr = {}
    O.step(x, f, 3, inp, O.Params(nx=40, ny=36, mdf_iters=40, marker_offset=0.5), trace=tr)
    mm = tr["mdf_mismatch"]
    assert all(b <= a * (1 + 1e-9) for a, b in zip(mm, mm[1:])), mm
    assert mm[-1] < 0.5 * mm[0], (mm[0], mm[-1])


def test_two_layer_reverse_mode_matches_central_differences():
    # L(x) = sum_c R_c . S2[v](c) + sum_i q_i . I2[u](x_i) for fixed random
    # R, v, u, q: its gradient in x only flows through the marker positions
    topo = O.Topology(np.array([0, 5, 6, 9]))      # a chain, a single node, a short chain
    p = O.Params(nx=16, ny=12, marker_offset=0.6)
    g = np.random.default_rng(3)
    x0 = torch.tensor(np.stack([g.uniform(2, 14, 9), g.uniform(2, 10, 9)]), dtype=DT)
    v = torch.tensor(g.normal(size=(2, 9)), dtype=DT)
    q = torch.tensor(g.normal(size=(2, 9)), dtype=DT)
    R = torch.tensor(g.normal(size=(2, 12, 16)), dtype=DT)
    u = torch.tensor(g.normal(size=(2, 12, 16)), dtype=DT)

    def L(x):
        return (O.spread2(x, v, topo, p) * R).sum() + (O.interpolate2(x, u, topo, p) * q).sum()

    x = x0.clone().requires_grad_(True)
    L(x).backward()
    grad = x.grad
    assert torch.isfinite(grad).all()
    h = 1e-6
    fd = torch.zeros_like(x0)
    for k in range(2):
        for i in range(9):
            e = torch.zeros_like(x0)
            e[k, i] = h
            fd[k, i] = (L(x0 + e) - L(x0 - e)) / (2 * h)
    assert torch.allclose(grad, fd, rtol=1e-6, atol=1e-7), float((grad - fd).abs().max())
    # the single node's own markers coincide with it: its gradient is the
    # one-layer transfers' gradient there
    assert float(grad[:, 5].abs().max()) > 0
