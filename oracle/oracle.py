"""FP64 CPU oracle of the Microcosmos filament-fluid timestep.

TEST INFRASTRUCTURE ONLY.  This module exists so that tests, the smoke check
and the benchmark's CPU baseline can check the HIP path against a plain,
slow, obviously correct implementation.  The product path never imports it.

Everything is plain PyTorch on the CPU in float64, written in the paper's
order and notation; every step that is elementwise over nodes, edges or cells
is written as one vectorised expression over the index set it ranges over.
Reverse mode (the gradient of a rollout with respect to the rest angles and
the initial positions) is PyTorch's autograd of exactly this forward code.

Readings where the paper is silent (stated once here, cited per function):
  * sub-step order within one step: actuation, elastic force, deposit,
    Gaussian filter, repulsion, force spread, fluid update, gather+integrate;
  * PBD couples to the fluid as an explicit immersed-boundary force: the
    projected positions y are the elastic target and F_el = k_el (y - x);
  * edge angles are re-synchronised to atan2 of the edge vectors at the start
    of every step; K PBD iterations; two-colour Gauss-Seidel ordering;
  * bend constraint angle difference wrapped into (-pi, pi];
  * particle/grid transfer with Peskin's 4-point kernel, cell centres at
    integer coordinates, periodic grid;
  * Gaussian filter sigma = 1 cell, radius 4, sampled taps normalised, circular
    (identical to the FFT convolution with the same kernel);
  * repulsion = -k_rep * interpolate(central difference of the filtered field);
  * D2Q9 two-relaxation-time collision with Guo forcing, magic parameter 1/4;
  * explicit Euler integration of nodes with the interpolated fluid velocity.

Pins: see tests/test_oracle_pins.py (closed forms, invariants, brute force,
library routines, physics).  Nothing here is "parity unpinned" except the
numeric constants of the reading (stiffnesses, k_el, k_rep, sigma), which the
paper does not give.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

DT = torch.float64
TWO_PI = 2.0 * math.pi


@dataclass
class Params:
    """Physical and numerical constants of one world (lattice units)."""

    nx: int
    ny: int
    tau: float = 1.0             # BGK-equivalent relaxation time, nu = (tau - 1/2)/3
    trt_magic: float = 0.25      # TRT magic parameter Lambda
    k_bend: float = 0.5          # bending stiffness (Eq. 1)
    k_stretch: float = 1.0       # stretch stiffness (Eq. 3)
    k_shear: float = 0.5         # shear blend (Eq. 3)
    pbd_iters: int = 4           # PBD iterations per step
    k_elastic: float = 0.05      # F_el = k_elastic (y - x)
    k_repulse: float = 0.1       # steric repulsion strength
    sigma: float = 1.0           # Gaussian filter width (cells)
    radius: int = 4              # Gaussian filter truncation radius (cells)
    u_max: float = 0.3           # Mach guard on |u|
    mdf_iters: int = 1           # multi-direct forcing iterations (1: explicit coupling)
    marker_offset: float = 0.0   # two-layer markers at +-offset along the normal (0: one layer)


# ---------------------------------------------------------------------------
# Filament topology (Methods, Filaments: filaments extend to loops and
# branches through a graph representation; Discussion: topologies are cactus
# graphs)
# ---------------------------------------------------------------------------

class Topology:
    """Index sets of a set of filaments given by CSR offsets.

    Open chain: edge e joins nodes (e, e+1) of one filament; joint i is an
    interior node, between edges i-1 and i.  Closed loop (``closed[f]``, at
    least three nodes): also the edge of the last node, which joins it to the
    first, and a joint at every node (the first node's joint is between the
    closing edge and edge 0).  Edges and joints are stored at the index of
    their node: edge e joins e and edge_next[e]; joint i is between edges
    joint_prev[i] and i.  Sets are split by the parity of the local index
    (edge: e - o_f; joint: i - o_f - 1 on chains, i - o_f on loops) for
    two-colour Gauss-Seidel sweeps; on a loop of odd length the last edge
    and the last joint (which meet the first ones) get a third colour.

    Branches (reading; the paper gives no equations for them): an open
    filament f with ``parent[f] = p >= 0`` hangs from node p of an earlier
    filament through an attachment edge from p to f's first node c0, with
    rest length ``attach[0, f]``, a joint at p between p's entering edge
    (prev[p]: p is a node of a loop or a non-first node of a chain) and the
    attachment edge (rest angle ``attach[1, f]``), and a joint at c0
    between the attachment edge and f's edge 0 (rest angle ``attach[2, f]``,
    if f has two nodes or more).  A node carries at most one attached
    filament, so every graph is a cactus of chains and loops whose branch
    points have degree three.  The attachment joints are not actuated; the
    attachment constraints use the world's scalar stiffnesses.
    """

    def __init__(self, fil_offset, closed=None, parent=None, attach=None):
        off = np.asarray(fil_offset, dtype=np.int64)
        self.fil_offset = off
        self.n_filaments = len(off) - 1
        self.n = int(off[-1])
        closed = np.zeros(self.n_filaments, dtype=bool) if closed is None else np.asarray(closed, dtype=bool)
        self.closed = closed
        edges, ecol, joints, jcol, jlocal, jfil, jcount = [], [], [], [], [], [], []
        nxt = np.arange(self.n, dtype=np.int64) + 1
        prv = np.arange(self.n, dtype=np.int64) - 1
        fil_of_node = np.zeros(self.n, dtype=np.int64)
        for f in range(self.n_filaments):
            a, b = int(off[f]), int(off[f + 1])
            n = b - a
            fil_of_node[a:b] = f
            ring = bool(closed[f]) and n >= 3
            for e in range(a, b if ring else b - 1):
                edges.append(e)
                k = e - a
                ecol.append(2 if (ring and n % 2 == 1 and k == n - 1) else k % 2)
            if ring:
                nxt[b - 1] = a
                prv[a] = b - 1
                for i in range(a, b):
                    k = i - a
                    joints.append(i)
                    jlocal.append(k)
                    jcol.append(2 if (n % 2 == 1 and k == n - 1) else k % 2)
                    jfil.append(f)
                    jcount.append(n)
            else:
                for i in range(a + 1, b - 1):
                    joints.append(i)
                    jlocal.append(i - a - 1)
                    jcol.append((i - a - 1) % 2)
                    jfil.append(f)
                    jcount.append(n - 2)
        t = lambda v: torch.tensor(v, dtype=torch.int64)
        self.edges = t(edges)
        self.edge_next = torch.from_numpy(nxt)
        self.joints = t(joints)
        self.joint_prev = torch.from_numpy(prv)
        self.joint_local = t(jlocal)
        self.joint_fil = t(jfil)
        self.joint_count = t(jcount)        # n_f - 2 for a chain's joint, n_f for a loop's
        self.fil_of_node = torch.from_numpy(fil_of_node)
        ec = np.array(ecol, dtype=np.int64)
        jc = np.array(jcol, dtype=np.int64)
        ed = np.array(edges, dtype=np.int64)
        jo = np.array(joints, dtype=np.int64)
        self.edge_sets = [t(ed[ec == c]) for c in range(3)]
        self.joint_sets = [t(jo[jc == c]) for c in range(3)]
        # attachments (branches), one per child filament, in filament order
        par = np.full(self.n_filaments, -1, dtype=np.int64) if parent is None else np.asarray(parent, np.int64)
        att = np.zeros((3, self.n_filaments)) if attach is None else np.asarray(attach, dtype=np.float64)
        kids = [f for f in range(self.n_filaments) if par[f] >= 0]
        used = set()
        for f in kids:
            pn = int(par[f])
            pf = int(fil_of_node[pn]) if 0 <= pn < self.n else -1
            if not 0 <= pf < f:
                raise ValueError(f"filament {f}: its parent node must lie in an earlier filament")
            if closed[f]:
                raise ValueError(f"filament {f}: a closed loop cannot hang from a parent node")
            ring_p = bool(closed[pf]) and off[pf + 1] - off[pf] >= 3
            if not ring_p and pn == off[pf]:
                raise ValueError(f"filament {f}: its parent node has no entering edge")
            if pn in used:
                raise ValueError(f"node {pn} carries two attached filaments")
            used.add(pn)
        kid = np.array(kids, dtype=np.int64)
        self.att_fil = t(kids)
        self.att_parent = t(par[kid])                      # node p
        self.att_child = t(off[kid])                       # node c0
        self.att_in = t(prv[par[kid]])                     # p's entering edge (its node index)
        self.att_length = torch.from_numpy(att[0, kid].copy())
        self.att_angle_parent = torch.from_numpy(att[1, kid].copy())
        self.att_angle_child = torch.from_numpy(att[2, kid].copy())
        has_edge0 = (off[kid + 1] - off[kid]) >= 2
        self.att_joint_child = t(kid[has_edge0].tolist())  # attachments with a joint at c0
        self.att_joint_child_idx = t(np.nonzero(has_edge0)[0].tolist())


# ---------------------------------------------------------------------------
# S0. Actuation: time-dependent rest angle (Experiments, Hand-designed
# locomotion: sinusoidal wave along the body; reading: one travelling
# wavelength per body)
# ---------------------------------------------------------------------------

def actuation(rest_angle, topo: Topology, amp, period, phase, t):
    """theta_hat_i = theta_rest_i + A_f sin(2 pi t / T_f + psi_f - 2 pi k / m_f), k the
    joint's local index, m_f its filament's joint count (n_f - 2; n_f on a loop)."""
    theta_hat = rest_angle.clone()
    if topo.joints.numel() == 0:
        return theta_hat
    f = topo.joint_fil
    arg = (TWO_PI * float(t) / period[f] + phase[f]
           - TWO_PI * topo.joint_local.to(DT) / topo.joint_count.to(DT))
    return theta_hat.index_add(0, topo.joints, amp[f] * torch.sin(arg))


# ---------------------------------------------------------------------------
# S1. Elastic force: PBD Cosserat projection (Methods, Bending Pass Eq. 1,
# Position Pass Eqs. 2-4)
# ---------------------------------------------------------------------------

def wrap_angle(d):
    """Map an angle difference into (-pi, pi]."""
    return d - TWO_PI * torch.ceil((d - math.pi) / TWO_PI)


def edge_angles(y, topo: Topology):
    """theta_e = atan2 of edge vector y_next(e) - y_e, for every edge (others 0)."""
    theta = torch.zeros(topo.n, dtype=DT)
    if topo.edges.numel() == 0:
        return theta
    e = topo.edges
    v = y[:, topo.edge_next[e]] - y[:, e]
    return theta.index_put((e,), torch.atan2(v[1], v[0]))


def _at(k, idx):
    """A stiffness: a scalar, or a per-node tensor read at the index set."""
    return k[idx] if torch.is_tensor(k) else k


def bend_pass(theta, joints, theta_hat, k_bend, prev=None):
    """Eq. 1 for a set of joints that share no edge: C = wrap(th_2 - th_1) - th_hat,
    th_1 += k C / 2, th_2 -= k C / 2, with th_1 the edge before the joint
    (prev[joint], default joint - 1).  k_bend: scalar or per joint (node)."""
    if joints.numel() == 0:
        return theta
    before = joints - 1 if prev is None else prev[joints]
    c = wrap_angle(theta[joints] - theta[before]) - theta_hat[joints]
    k = _at(k_bend, joints)
    return theta.index_add(0, before, 0.5 * k * c).index_add(0, joints, -0.5 * k * c)


def position_pass(y, theta, edges, rest_length, k_stretch, k_shear, nxt=None):
    """Eqs. 2-4 for a set of edges that share no node; edge e joins e and
    nxt[e] (default e + 1).  k_stretch, k_shear: scalars or per edge (node)."""
    if edges.numel() == 0:
        return y
    other = edges + 1 if nxt is None else nxt[edges]
    v = y[:, other] - y[:, edges]
    ell = torch.sqrt(v[0] * v[0] + v[1] * v[1])
    L = rest_length[edges]
    ks, ksh = _at(k_stretch, edges), _at(k_shear, edges)
    c_stretch = (ell - L) * v / ell                                          # Eq. 2
    d = torch.stack([torch.cos(theta[edges]), torch.sin(theta[edges])])
    dx = 0.5 * ks * (c_stretch + ksh * (v - L * d - c_stretch))              # Eq. 3
    return y.index_add(1, edges, dx).index_add(1, other, -dx)               # Eq. 4


def attachment_angles(y, topo: Topology):
    """Angle of every attachment edge p -> c0."""
    v = y[:, topo.att_child] - y[:, topo.att_parent]
    return torch.atan2(v[1], v[0])


def bend_attachments(theta, th_att, topo: Topology, k_bend):
    """Eq. 1 at the attachment joints: first at every parent node (edges:
    p's entering edge, then the attachment edge), then at every child's
    first node (the attachment edge, then the child's edge 0)."""
    if topo.att_parent.numel() == 0:
        return theta, th_att
    a = topo.att_in
    c = wrap_angle(th_att - theta[a]) - topo.att_angle_parent
    theta = theta.index_add(0, a, 0.5 * k_bend * c)
    th_att = th_att - 0.5 * k_bend * c
    i, e = topo.att_joint_child_idx, topo.att_child[topo.att_joint_child_idx]
    if i.numel():
        c = wrap_angle(theta[e] - th_att[i]) - topo.att_angle_child[i]
        th_att = th_att.index_add(0, i, 0.5 * k_bend * c)
        theta = theta.index_add(0, e, -0.5 * k_bend * c)
    return theta, th_att


def position_attachments(y, th_att, topo: Topology, k_stretch, k_shear):
    """Eqs. 2-4 on every attachment edge p -> c0."""
    if topo.att_parent.numel() == 0:
        return y
    a, b = topo.att_parent, topo.att_child
    v = y[:, b] - y[:, a]
    ell = torch.sqrt(v[0] * v[0] + v[1] * v[1])
    L = topo.att_length
    c_stretch = (ell - L) * v / ell
    d = torch.stack([torch.cos(th_att), torch.sin(th_att)])
    dx = 0.5 * k_stretch * (c_stretch + k_shear * (v - L * d - c_stretch))
    return y.index_add(1, a, dx).index_add(1, b, -dx)


def pbd_project(x, topo: Topology, theta_hat, rest_length, p: Params, iters=None, stiff=None):
    """K iterations of (bend: colours 0, 1, 2, then the attachment joints;
    position: colours 0, 1, 2, then the attachment edges) from y = x.

    ``stiff``: optional per-node (k_bend, k_stretch, k_shear) tensors (the
    paper's per-edge stiffnesses), else the scalars of p (the attachments
    always take the scalars).  Returns the projected positions y and the
    edge angles theta."""
    iters = p.pbd_iters if iters is None else iters
    kb, ks, ksh = (p.k_bend, p.k_stretch, p.k_shear) if stiff is None else stiff
    y = x
    theta = edge_angles(y, topo)
    th_att = attachment_angles(y, topo)
    for _ in range(iters):
        for js in topo.joint_sets:
            theta = bend_pass(theta, js, theta_hat, kb, topo.joint_prev)
        theta, th_att = bend_attachments(theta, th_att, topo, p.k_bend)
        for es in topo.edge_sets:
            y = position_pass(y, theta, es, rest_length, ks, ksh, topo.edge_next)
        y = position_attachments(y, th_att, topo, p.k_stretch, p.k_shear)
    return y, theta


def elastic_force(x, topo: Topology, theta_hat, rest_length, p: Params, stiff=None):
    """F_el,i = k_el (y_i - x_i) with y the PBD projection of x."""
    y, _ = pbd_project(x, topo, theta_hat, rest_length, p, stiff=stiff)
    return p.k_elastic * (y - x)


# ---------------------------------------------------------------------------
# Energy field (Methods, Fields: a persistent scalar field of Gaussian packets
# at random positions, a chemotaxis target; Experiments, Neuroevolution of
# Controller Circuit: each node senses the energy at its position, fitness
# adds the total energy collected).  Reading: packets are Gaussians summed
# into every cell (minimum image); at every step each node senses
# e_i = I[E](x_i) with the transfer kernel at the step's starting position,
# collects c_i = rate e_i, which is taken out of the field by the same kernel
# (E <- E - S[c], so the field loses exactly what the nodes collect), and the
# filament's collected total grows by the sum of its nodes' c_i.  The field
# does not act on the motion.
# ---------------------------------------------------------------------------

def energy_packets(nx, ny, centres, amps, widths):
    """E_c = sum_p A_p exp(-|c - c_p|^2 / (2 s_p^2)) over every cell (minimum
    image); centres [2, P], amps [P], widths [P]."""
    cx = torch.arange(nx, dtype=DT)
    cy = torch.arange(ny, dtype=DT)
    E = torch.zeros(ny, nx, dtype=DT)
    for k in range(centres.shape[1]):
        dx = min_image(cx - centres[0, k], nx)
        dy = min_image(cy - centres[1, k], ny)
        r2 = dy[:, None] ** 2 + dx[None, :] ** 2
        E = E + amps[k] * torch.exp(-r2 / (2.0 * widths[k] ** 2))
    return E


def energy_update(x, E, topo: Topology, rate, p: Params):
    """One step of sensing and collection at positions x: returns the sensed
    values e [N], the energy collected per filament [F] and the field after
    collection."""
    e = interpolate(x, E[None], p)[0]
    c = rate * e
    collected = torch.zeros(topo.n_filaments, dtype=DT).index_add(0, topo.fil_of_node, c)
    return e, collected, E - spread(x, c[None], p)[0]


# ---------------------------------------------------------------------------
# Behavioural descriptors of the quality-diversity search (Experiments, QD
# Search, Eqs. 5-6): bending effort E_bend = sum |theta_rest^{t-1} -
# theta_rest^t|^2 and stretching effort E_pos = sum |L_rest^{t-1} -
# L_rest^t|^2, per filament, for one change of the rest values (a controller
# writing new ones); summed over the filament's joints and edges.
# ---------------------------------------------------------------------------

def rest_effort(topo: Topology, old_angle, new_angle, old_length, new_length):
    """(E_bend, E_pos) per filament [2, F] for one change of the rest values."""
    F = topo.n_filaments
    eb = torch.zeros(F, dtype=DT).index_add(
        0, topo.joint_fil, (old_angle[topo.joints] - new_angle[topo.joints]) ** 2)
    ep = torch.zeros(F, dtype=DT).index_add(
        0, topo.fil_of_node[topo.edges], (old_length[topo.edges] - new_length[topo.edges]) ** 2)
    return torch.stack([eb, ep])


# ---------------------------------------------------------------------------
# Particle <-> grid transfer (Methods, Fluid-filament interaction: immersed
# boundary with a smoothing kernel over a small neighbourhood; reading:
# Peskin's 4-point function)
# ---------------------------------------------------------------------------

def peskin_phi(r):
    """Peskin's 4-point regularised delta function (one dimension).

    phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4r^2)) / 8       for |r| <= 1
           = (5 - 2|r| - sqrt(-7 + 12|r| - 4r^2)) / 8     for 1 <= |r| <= 2
           = 0                                              otherwise
    Each branch is evaluated on |r| clamped to its own interval so that no
    square root ever sees a negative argument (keeps reverse mode finite).
    """
    a = torch.abs(r)
    ai = torch.clamp(a, max=1.0)
    ao = torch.clamp(a, min=1.0, max=2.0)
    inner = (3.0 - 2.0 * ai + torch.sqrt(1.0 + 4.0 * ai - 4.0 * ai * ai)) / 8.0
    outer = (5.0 - 2.0 * ao - torch.sqrt(-7.0 + 12.0 * ao - 4.0 * ao * ao)) / 8.0
    return torch.where(a <= 1.0, inner, torch.where(a < 2.0, outer, torch.zeros_like(a)))


def support(xc, n):
    """Cells floor(x)-1 .. floor(x)+2 (mod n) and their 1D weights phi(c - x): [N, 4] each."""
    base = torch.floor(xc.detach())
    m = torch.arange(-1, 3, dtype=DT)
    cells = base[:, None] + m[None, :]
    w = peskin_phi(cells - xc[:, None])
    idx = torch.remainder(cells.to(torch.int64), n)
    return idx, w


def transfer_stencil(x, p: Params):
    """Flat cell indices [N, 16] and weights W(c - x_i) = phi(dx) phi(dy) [N, 16]."""
    ix, wx = support(x[0], p.nx)
    iy, wy = support(x[1], p.ny)
    flat = (iy[:, :, None] * p.nx + ix[:, None, :]).reshape(-1, 16)
    w = (wy[:, :, None] * wx[:, None, :]).reshape(-1, 16)
    return flat, w


def spread(x, vals, p: Params):
    """Grid field G_c = sum_i W(c - x_i) v_i for vals [C, N] -> [C, ny, nx]."""
    flat, w = transfer_stencil(x, p)
    C = vals.shape[0]
    out = []
    for k in range(C):
        g = torch.zeros(p.ny * p.nx, dtype=DT)
        g = g.index_add(0, flat.reshape(-1), (w * vals[k][:, None]).reshape(-1))
        out.append(g.reshape(p.ny, p.nx))
    return torch.stack(out)


def interpolate(x, field, p: Params):
    """Node values v_i = sum_c W(c - x_i) G_c for field [C, ny, nx] -> [C, N]."""
    flat, w = transfer_stencil(x, p)
    return torch.stack([(field[k].reshape(-1)[flat] * w).sum(dim=1) for k in range(field.shape[0])])


# ---------------------------------------------------------------------------
# Leakage fixes of the coupling (Methods, Fluid-filament Interaction: Multi-
# Direct Forcing, and broadcasting the filament as a two-layer version of
# itself).  Reading:
#   * two layers: node i is broadcast as two markers X_i = x_i +- delta n_i
#     (n_i the unit normal: the tangent is x_next - x_prev where the node has
#     two neighbours, the edge direction at a chain end); spreading gives each
#     marker half of the node's value, and a node samples the mean of its two
#     markers' interpolated values; delta = 0 is the one-layer transfer;
#   * MDF: the node's desired velocity is what the explicit coupling gives it,
#     U_d = I2[u*] + F / 2 with u* = j / rho (the fluid velocity without the
#     body force) and F the node force (the Guo half-force gain, rho_0 = 1);
#     the first iteration spreads F itself; each further one samples
#     u = (j + F_grid / 2) / rho at the markers and spreads the correction
#     2 (U_d - I2[u]).  One iteration is the explicit coupling.
# ---------------------------------------------------------------------------

def marker_normals(x, topo: Topology):
    """Unit normal (-t_y, t_x) at every node from its neighbours (zero for a
    single-node filament)."""
    N = topo.n
    nxt = torch.arange(N) + 1
    prv = torch.arange(N) - 1
    has_next = torch.zeros(N, dtype=torch.bool)
    has_prev = torch.zeros(N, dtype=torch.bool)
    if topo.edges.numel():
        e = topo.edges
        nxt = nxt.index_put((e,), topo.edge_next[e])
        has_next[e] = True
        prv = prv.index_put((topo.edge_next[e],), e)
        has_prev[topo.edge_next[e]] = True
    i = torch.arange(N)
    a = torch.where(has_prev, prv, i)
    b = torch.where(has_next, nxt, i)
    t = x[:, b.clamp(0, max(N - 1, 0))] - x[:, a.clamp(0, max(N - 1, 0))]
    n2 = t[0] ** 2 + t[1] ** 2
    # the square root of a masked length, so that a node without a tangent
    # (its normal is zero) also has a zero derivative rather than 0 * inf
    safe = torch.sqrt(torch.where(n2 > 0, n2, torch.ones_like(n2)))
    t = torch.where(n2 > 0, t / safe, torch.zeros_like(t))
    return torch.stack([-t[1], t[0]])


def spread2(x, vals, topo: Topology, p: Params):
    """Two-layer spread: half of each node's value from each of its markers."""
    if p.marker_offset == 0.0:
        return spread(x, vals, p)
    d = p.marker_offset * marker_normals(x, topo)
    return 0.5 * (spread(x + d, vals, p) + spread(x - d, vals, p))


def interpolate2(x, field, topo: Topology, p: Params):
    """Two-layer interpolation: the mean of the node's two markers' values."""
    if p.marker_offset == 0.0:
        return interpolate(x, field, p)
    d = p.marker_offset * marker_normals(x, topo)
    return 0.5 * (interpolate(x + d, field, p) + interpolate(x - d, field, p))


def coupling_force(x, f, force, topo: Topology, p: Params, trace=None):
    """Grid force of the step: the node forces spread (two-layer), then
    mdf_iters - 1 multi-direct-forcing corrections."""
    Fg = spread2(x, force, topo, p)
    if p.mdf_iters <= 1:
        return Fg
    cx = C_Q[:, 0].reshape(9, 1, 1)
    cy = C_Q[:, 1].reshape(9, 1, 1)
    rho = f.sum(dim=0)
    j = torch.stack([(f * cx).sum(dim=0), (f * cy).sum(dim=0)])
    U_d = interpolate2(x, j / rho, topo, p) + 0.5 * force
    mismatch = []
    for _ in range(p.mdf_iters - 1):
        U = interpolate2(x, (j + 0.5 * Fg) / rho, topo, p)
        mismatch.append(float((U_d - U).detach().abs().max()))
        Fg = Fg + spread2(x, 2.0 * (U_d - U), topo, p)
    if trace is not None:
        trace["mdf_mismatch"] = mismatch
        trace["U_d"] = U_d
    return Fg


# ---------------------------------------------------------------------------
# S2-S4. Steric repulsion field (Methods, Fields: deposit, Gaussian filter,
# gradient of the density gives repulsion)
# ---------------------------------------------------------------------------

def deposit(x, p: Params):
    """s_c = sum_i W(c - x_i)."""
    ones = torch.ones((1, x.shape[1]), dtype=DT)
    return spread(x, ones, p)[0]


def gaussian_taps(sigma, radius):
    k = torch.arange(-radius, radius + 1, dtype=DT)
    g = torch.exp(-k * k / (2.0 * sigma * sigma))
    return g / g.sum()


def gaussian_filter(s, p: Params):
    """Circular separable convolution: first along x, then along y."""
    g = gaussian_taps(p.sigma, p.radius)
    R = p.radius
    tx = sum(g[k + R] * torch.roll(s, shifts=k, dims=1) for k in range(-R, R + 1))
    return sum(g[k + R] * torch.roll(tx, shifts=k, dims=0) for k in range(-R, R + 1))


def central_difference(st):
    """(D s)_c = ((s[x+1] - s[x-1]) / 2, (s[y+1] - s[y-1]) / 2), periodic; [2, ny, nx]."""
    gx = 0.5 * (torch.roll(st, shifts=-1, dims=1) - torch.roll(st, shifts=1, dims=1))
    gy = 0.5 * (torch.roll(st, shifts=-1, dims=0) - torch.roll(st, shifts=1, dims=0))
    return torch.stack([gx, gy])


def repulsion(x, st, p: Params):
    """F_rep,i = -k_rep sum_c W(c - x_i) (D s~)_c."""
    return -p.k_repulse * interpolate(x, central_difference(st), p)


# ---------------------------------------------------------------------------
# S6. Fluid: D2Q9 lattice Boltzmann, TRT collision with Guo forcing, periodic
# streaming (Methods, Fields; Fluid-filament interaction)
# ---------------------------------------------------------------------------

# D2Q9 velocities, weights and opposite directions (Qian, d'Humieres, Lallemand)
C_Q = torch.tensor([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
                   dtype=DT)
W_Q = torch.tensor([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=DT)
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def lbm_collide(f, F, p: Params):
    """TRT collision with Guo forcing at every cell.

    f: [9, ny, nx] pre-collision populations; F: [2, ny, nx] body force.
    Returns (post-collision populations, u) with u = (sum_q f_q c_q + F/2) / rho.
    """
    cx = C_Q[:, 0].reshape(9, 1, 1)
    cy = C_Q[:, 1].reshape(9, 1, 1)
    w = W_Q.reshape(9, 1, 1)
    rho = f.sum(dim=0)
    ux = ((f * cx).sum(dim=0) + 0.5 * F[0]) / rho
    uy = ((f * cy).sum(dim=0) + 0.5 * F[1]) / rho
    cu = cx * ux + cy * uy
    usq = ux * ux + uy * uy
    feq = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)
    S = w * ((3.0 * (cx - ux) + 9.0 * cu * cx) * F[0] + (3.0 * (cy - uy) + 9.0 * cu * cy) * F[1])
    om_p = 1.0 / p.tau
    om_m = 1.0 / (p.trt_magic / (p.tau - 0.5) + 0.5)
    opp = OPP
    sym = lambda a: 0.5 * (a + a[opp])
    anti = lambda a: 0.5 * (a - a[opp])
    fstar = (f - om_p * (sym(f) - sym(feq)) - om_m * (anti(f) - anti(feq))
             + (1.0 - 0.5 * om_p) * sym(S) + (1.0 - 0.5 * om_m) * anti(S))
    return fstar, torch.stack([ux, uy])


def lbm_stream(fstar):
    """f_q(c + c_q) <- f*_q(c), periodic."""
    return torch.stack([torch.roll(fstar[q], shifts=(int(C_Q[q, 1]), int(C_Q[q, 0])), dims=(0, 1))
                        for q in range(9)])


def rest_populations(p: Params):
    """Fluid at rest: f_q = w_q (rho = 1, u = 0)."""
    return W_Q.reshape(9, 1, 1).expand(9, p.ny, p.nx).clone()


# ---------------------------------------------------------------------------
# One step and rollouts
# ---------------------------------------------------------------------------

@dataclass
class Inputs:
    """Fixed per-world arrays (float64 / int64 tensors)."""

    topo: Topology
    rest_angle: torch.Tensor
    rest_length: torch.Tensor
    amp: torch.Tensor
    period: torch.Tensor
    phase: torch.Tensor
    stiff: tuple = None          # per-node (k_bend, k_stretch, k_shear), or None: Params scalars


def inputs_from_world(w) -> Inputs:
    """Widen a workloads.World to float64 tensors (exact)."""
    t = lambda a: torch.from_numpy(np.asarray(a).astype(np.float64))
    stiff = getattr(w, "stiffness", None)
    return Inputs(
        topo=Topology(w.fil_offset, getattr(w, "closed", None), getattr(w, "parent", None),
                      getattr(w, "attach", None)),
        rest_angle=t(w.rest_angle),
        rest_length=t(w.rest_length),
        amp=t(w.act_amp),
        period=t(w.act_period),
        phase=t(w.act_phase),
        stiff=None if stiff is None else tuple(t(k) for k in stiff),
    )


def positions_from_world(w):
    return torch.from_numpy(w.cell.astype(np.float64) + w.frac.astype(np.float64))


def step(x, f, t, inp: Inputs, p: Params, rest_angle=None, trace=None):
    """Advance (x, f) by one step at time index t; returns (x', f', u_t).

    ``rest_angle`` overrides inp.rest_angle (for differentiation).  If ``trace``
    is a dict, intermediate fields are stored in it.
    """
    ra = inp.rest_angle if rest_angle is None else rest_angle
    theta_hat = actuation(ra, inp.topo, inp.amp, inp.period, inp.phase, t)      # S0
    f_el = elastic_force(x, inp.topo, theta_hat, inp.rest_length, p, inp.stiff)  # S1
    s = deposit(x, p)                                                           # S2
    st = gaussian_filter(s, p)                                                  # S3
    f_rep = repulsion(x, st, p)                                                 # S4
    force = f_el + f_rep
    Fg = coupling_force(x, f, force, inp.topo, p, trace)                        # S5
    fstar, u = lbm_collide(f, Fg, p)                                            # S6
    f_new = lbm_stream(fstar)
    x_new = x + interpolate2(x, u, inp.topo, p)                                 # S7
    if trace is not None:
        trace.update(theta_hat=theta_hat, f_el=f_el, s=s, st=st, f_rep=f_rep, force=force,
                     Fg=Fg, u=u, fstar=fstar)
    return x_new, f_new, u


def rollout(x, f, t0, n, inp: Inputs, p: Params, rest_angle=None, every=None):
    """n steps from time t0.  ``every(k, x, f, u)`` is called after step k (0-based)."""
    for k in range(n):
        x, f, u = step(x, f, t0 + k, inp, p, rest_angle=rest_angle)
        if every is not None:
            every(k, x, f, u)
    return x, f


def fold_loss(x, target):
    """Mean over nodes of the squared distance to the target: (1/N) sum_i |x_i - y*_i|^2."""
    return ((x - target) ** 2).sum() / x.shape[1]


def rollout_gradient(x0, f0, t0, n, inp: Inputs, p: Params, grad_xT, segment=20):
    """d(<grad_xT, x_T>)/d(rest_angle) and d/d(x0) by reverse mode over segments.

    The forward is replayed from the stored segment-start states (x, f); the
    adjoint of each segment is PyTorch's autograd of the forward code above.
    """
    starts = []
    x, f = x0.detach(), f0.detach()
    k = 0
    while k < n:
        starts.append((k, x, f))
        m = min(segment, n - k)
        with torch.no_grad():
            x, f = rollout(x, f, t0 + k, m, inp, p)
        k += m
    gx = grad_xT.detach().clone()
    gf = torch.zeros_like(f0)
    g_ra = torch.zeros_like(inp.rest_angle)
    for (k, xs, fs) in reversed(starts):
        m = min(segment, n - k)
        xs = xs.clone().requires_grad_(True)
        fs = fs.clone().requires_grad_(True)
        ra = inp.rest_angle.clone().requires_grad_(True)
        xe, fe = rollout(xs, fs, t0 + k, m, inp, p, rest_angle=ra)
        outs = [xe, fe]
        gouts = [gx, gf]
        gxs, gfs, gra = torch.autograd.grad(outs, [xs, fs, ra], gouts, allow_unused=True)
        gx = gxs.detach()
        gf = gfs.detach() if gfs is not None else torch.zeros_like(f0)
        if gra is not None:
            g_ra = g_ra + gra.detach()
    return g_ra, gx


# ---------------------------------------------------------------------------
# Folding objective (Experiments, Filament Folding): mean squared error
# between the Gaussian-splatted node density at the final step and a target
# image.  Reading: the image covers the periodic world; pixel (a, b) of a
# W x H image is centred at world point (-1/2 + (a + 1/2) nx / W,
# -1/2 + (b + 1/2) ny / H) (cells are centred at integer coordinates); node i
# adds amp * exp(-r^2 / (2 sigma^2)) to every pixel whose centre lies within
# r <= 5 sigma of it (periodic minimum-image distance, sigma in cells).
# ---------------------------------------------------------------------------

SPLAT_CUTOFF = 5.0      # truncation radius in units of sigma


def pixel_centres(nx, ny, width, height):
    """World coordinates of the pixel centres along x (width) and y (height)."""
    cx = -0.5 + (torch.arange(width, dtype=DT) + 0.5) * (nx / width)
    cy = -0.5 + (torch.arange(height, dtype=DT) + 0.5) * (ny / height)
    return cx, cy


def min_image(d, n):
    """Periodic difference d reduced to [-n/2, n/2)."""
    return d - n * torch.floor(d / n + 0.5)


def density_image(x, nx, ny, width, height, sigma, amp=1.0):
    """Gaussian-splatted density image [height, width] of nodes x [2, N]
    (every node against every pixel, then the cutoff)."""
    cx, cy = pixel_centres(nx, ny, width, height)
    dx = min_image(x[0][:, None, None] - cx[None, None, :], nx)      # [N, 1, W]
    dy = min_image(x[1][:, None, None] - cy[None, :, None], ny)      # [N, H, 1]
    r2 = dx * dx + dy * dy                                           # [N, H, W]
    g = amp * torch.exp(-r2 / (2.0 * sigma * sigma))
    g = torch.where(r2 <= (SPLAT_CUTOFF * sigma) ** 2, g, torch.zeros_like(g))
    return g.sum(dim=0)


def density_loss(image, target):
    """Mean over pixels of the squared difference to the target image."""
    return ((image - target) ** 2).mean()
