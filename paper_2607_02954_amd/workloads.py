"""Seeded synthetic inputs for the filament-fluid timestep.

This module is the one piece shared by the GPU path and the FP64 oracle.  It
only draws random numbers and lays out the initial state (straight chains,
rest shapes, actuation parameters, loss targets); it contains none of the
method's arithmetic (no forces, no transfer kernel, no fluid update).

Workloads follow the paper's setting (Methods, "Filaments": chains of nodes
with per-edge rest length and per-joint rest angle; "Fields": a periodic 2D
grid) with sizes of the scaling, folding and population experiments
(Experiments, "Scalability", "Filament Folding").  Every array is produced by
numpy's PCG64 generator from an integer seed.

Positions are handed out as an integer cell plus a float32 fraction in
[0, 1); the exact real position is ``cell + float64(frac)``, so both sides
start from bit-identical coordinates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class World:
    """Initial state of one world (host numpy arrays)."""

    nx: int
    ny: int
    fil_offset: np.ndarray          # int32 [F+1], CSR offsets into the node arrays
    cell: np.ndarray                # int32 [2, N] integer cell of every node (x row, y row)
    frac: np.ndarray                # float32 [2, N] fractional part, in [0, 1)
    rest_angle: np.ndarray          # float32 [N], joint at interior node i (edges i-1, i)
    rest_length: np.ndarray         # float32 [N], edge (i, i+1); last node of a filament unused
    act_amp: np.ndarray             # float32 [F] actuation amplitude (rad)
    act_period: np.ndarray          # float32 [F] actuation period (steps)
    act_phase: np.ndarray           # float32 [F] actuation phase offset (rad)
    target: Optional[np.ndarray] = None   # float64 [2, N] loss target (folding workload)
    meta: dict = field(default_factory=dict)
    stiffness: Optional[tuple] = None     # float32 [N] x 3: per-edge (k_bend, k_stretch, k_shear)
    closed: Optional[np.ndarray] = None   # bool [F]: filament f is a closed loop
    energy: Optional[np.ndarray] = None   # float32 [ny, nx] initial energy field
    parent: Optional[np.ndarray] = None   # int32 [F]: node filament f hangs from (-1: none)
    attach: Optional[np.ndarray] = None   # float [3, F]: attachment rest length, angle at the parent, angle at c0

    @property
    def n_particles(self) -> int:
        return int(self.fil_offset[-1])

    @property
    def n_filaments(self) -> int:
        return int(self.fil_offset.shape[0] - 1)

    def positions64(self) -> np.ndarray:
        """Exact node positions as float64 [2, N]."""
        return self.cell.astype(np.float64) + self.frac.astype(np.float64)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def split_position(x: np.ndarray):
    """Split float64 positions into (int32 cell, float32 frac) with frac in [0, 1)."""
    cell = np.floor(x).astype(np.int64)
    frac = (x - cell).astype(np.float32)
    roll = frac >= np.float32(1.0)
    cell = np.where(roll, cell + 1, cell)
    frac = np.where(roll, np.float32(0.0), frac).astype(np.float32)
    return cell.astype(np.int32), frac


def straight_chain(n: int, centre, angle: float, bond: float = 1.0) -> np.ndarray:
    """Nodes of a straight chain of ``n`` nodes, spacing ``bond``, float64 [2, n]."""
    s = (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * bond
    return np.stack([centre[0] + s * math.cos(angle), centre[1] + s * math.sin(angle)])


def _assemble(nx, ny, chains, rest_angle, rest_length, amp, period, phase, target=None, meta=None):
    lengths = [c.shape[1] for c in chains]
    off = np.zeros(len(chains) + 1, dtype=np.int32)
    off[1:] = np.cumsum(lengths)
    x = np.concatenate(chains, axis=1) if chains else np.zeros((2, 0))
    cell, frac = split_position(x)
    return World(
        nx=int(nx), ny=int(ny), fil_offset=off, cell=cell, frac=frac,
        rest_angle=np.asarray(rest_angle, dtype=np.float32),
        rest_length=np.asarray(rest_length, dtype=np.float32),
        act_amp=np.asarray(amp, dtype=np.float32),
        act_period=np.asarray(period, dtype=np.float32),
        act_phase=np.asarray(phase, dtype=np.float32),
        target=target, meta=dict(meta or {}))


def random_world(seed: int, nx: int, ny: int, lengths: List[int], *, angle_sd: float = 0.3,
                 amp: float = 0.0, period_range=(20.0, 100.0), bond: float = 1.0) -> World:
    """Chains of the given lengths, centres uniform in the box, orientations uniform.

    Rest angles ~ N(0, angle_sd^2) at interior joints; rest lengths = ``bond``.
    Actuation amplitude ``amp`` (0 disables it), period ~ U(period_range) steps,
    phase ~ U(0, 2 pi).
    """
    g = _rng(seed)
    F = len(lengths)
    centres = g.uniform(0.0, 1.0, size=(F, 2)) * np.array([nx, ny], dtype=np.float64)
    orient = g.uniform(0.0, 2.0 * math.pi, size=F)
    chains = [straight_chain(n, centres[f], orient[f], bond) for f, n in enumerate(lengths)]
    N = int(sum(lengths))
    rest_angle = np.zeros(N, dtype=np.float64)
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    draws = g.normal(0.0, angle_sd, size=N)
    for f in range(F):
        a, b = off[f], off[f + 1]
        if b - a >= 3:
            rest_angle[a + 1:b - 1] = draws[a + 1:b - 1]
    rest_length = np.full(N, bond, dtype=np.float64)
    period = g.uniform(period_range[0], period_range[1], size=F)
    phase = g.uniform(0.0, 2.0 * math.pi, size=F)
    amps = np.full(F, amp, dtype=np.float64)
    return _assemble(nx, ny, chains, rest_angle, rest_length, amps, period, phase,
                     meta=dict(seed=seed, orient=orient, centres=centres))


def polygon_loop(n: int, centre, angle: float = 0.0, bond: float = 1.0) -> np.ndarray:
    """Nodes of a regular n-gon with sides ``bond``, float64 [2, n]."""
    r = 0.5 * bond / math.sin(math.pi / n)
    a = angle + 2.0 * math.pi * np.arange(n) / n
    return np.stack([centre[0] + r * np.cos(a), centre[1] + r * np.sin(a)])


def generality_world(seed: int, nx: int, ny: int, chain_lengths: List[int], loop_lengths: List[int], *,
                     amp: float = 0.5, angle_sd: float = 0.3, stiffness_range=(0.2, 1.0)) -> World:
    """Open chains and closed loops with per-edge stiffnesses: chains as in
    random_world; loops are regular polygons (unit sides) with rest angles
    2 pi / n + N(0, angle_sd^2) at every node; every node's k_bend,
    k_stretch and k_shear ~ U(stiffness_range)."""
    g = _rng(seed + 32452843)
    base = random_world(seed, nx, ny, chain_lengths, angle_sd=angle_sd, amp=amp)
    chains = [base.positions64()[:, base.fil_offset[f]:base.fil_offset[f + 1]] for f in range(base.n_filaments)]
    ra = [base.rest_angle.astype(np.float64)]
    for n in loop_lengths:
        centre = g.uniform(0.0, 1.0, size=2) * np.array([nx, ny])
        chains.append(polygon_loop(n, centre, g.uniform(0, 2 * math.pi)))
        ra.append(2 * math.pi / n + g.normal(0.0, angle_sd, size=n))
    F = len(chains)
    N = sum(c.shape[1] for c in chains)
    amps = np.full(F, amp)
    period = np.concatenate([base.act_period, g.uniform(20.0, 100.0, size=len(loop_lengths))])
    phase = np.concatenate([base.act_phase, g.uniform(0.0, 2 * math.pi, size=len(loop_lengths))])
    w = _assemble(nx, ny, chains, np.concatenate(ra), np.ones(N), amps, period, phase,
                  meta=dict(seed=seed, name="generality"))
    w.closed = np.array([False] * len(chain_lengths) + [True] * len(loop_lengths))
    lo, hi = stiffness_range
    w.stiffness = tuple(g.uniform(lo, hi, size=N).astype(np.float32) for _ in range(3))
    return w


def branched_world(seed: int, nx: int, ny: int, n_creatures: int, *, amp: float = 0.5, loop_share: float = 0.3,
                   angle_sd: float = 0.3, max_children: int = 3) -> World:
    """Branched creatures (cactus graphs): a root filament (a chain of U{8..40}
    nodes, or with probability ``loop_share`` a regular polygon loop of
    U{6..16} unit sides) with 1..max_children chains of U{2..16} nodes hanging
    from distinct nodes that have an entering edge (a loop's nodes, a chain's
    non-first nodes), one of which may carry a grandchild chain.  Attachment
    rest length U(0.8, 1.2), rest angle at the parent +-U(0.6, 1.4), at the
    child's first node N(0, 0.2^2); each child starts straight along its
    attachment's rest direction.  Regular rest angles as random_world (loops:
    2 pi / n + noise); actuation amplitude ``amp`` on every filament."""
    g = _rng(seed + 15485863)
    chains, ra, closed, parent, attach = [], [], [], [], []
    n_nodes = 0
    for _ in range(n_creatures):
        centre = g.uniform(0.0, 1.0, size=2) * np.array([nx, ny])
        first = len(chains)
        if g.uniform() < loop_share:
            n = int(g.integers(6, 17))
            x = polygon_loop(n, centre, g.uniform(0, 2 * math.pi))
            chains.append(x)
            ra.append(2 * math.pi / n + g.normal(0.0, angle_sd, size=n))
            closed.append(True)
        else:
            n = int(g.integers(8, 41))
            x = straight_chain(n, centre, g.uniform(0, 2 * math.pi))
            chains.append(x)
            r = np.zeros(n)
            r[1:n - 1] = g.normal(0.0, angle_sd, size=n - 2)
            ra.append(r)
            closed.append(False)
        parent.append(-1)
        attach.append((0.0, 0.0, 0.0))
        # candidate parent nodes: (global index, position, entering-edge angle)
        def candidates(fi):
            xs = chains[fi]
            m = xs.shape[1]
            off = n_nodes + sum(c.shape[1] for c in chains[first:fi])
            out = []
            for k in range(m):
                if closed[fi]:
                    prev = xs[:, k - 1]
                elif k == 0:
                    continue
                else:
                    prev = xs[:, k - 1]
                d = xs[:, k] - prev
                out.append((off + k, xs[:, k], math.atan2(d[1], d[0])))
            return out
        used = set()
        kids = int(g.integers(1, max_children + 1))
        for c in range(kids):
            host = first if c == 0 or g.uniform() < 0.7 else len(chains) - 1
            cand = [q for q in candidates(host) if q[0] not in used]
            if not cand:
                continue
            node, pos, th_in = cand[int(g.integers(len(cand)))]
            used.add(node)
            La = g.uniform(0.8, 1.2)
            al = g.choice([-1.0, 1.0]) * g.uniform(0.6, 1.4)
            be = g.normal(0.0, 0.2)
            m = int(g.integers(2, 17))
            a0 = th_in + al
            c0 = pos + La * np.array([math.cos(a0), math.sin(a0)])
            a1 = a0 + be
            xs = np.stack([c0[0] + np.arange(m) * math.cos(a1), c0[1] + np.arange(m) * math.sin(a1)])
            chains.append(xs)
            r = np.zeros(m)
            if m >= 3:
                r[1:m - 1] = g.normal(0.0, angle_sd, size=m - 2)
            ra.append(r)
            closed.append(False)
            parent.append(node)
            attach.append((La, al, be))
        n_nodes += sum(c.shape[1] for c in chains[first:])
    F = len(chains)
    N = sum(c.shape[1] for c in chains)
    period = g.uniform(20.0, 100.0, size=F)
    phase = g.uniform(0.0, 2 * math.pi, size=F)
    w = _assemble(nx, ny, chains, np.concatenate(ra), np.ones(N), np.full(F, amp),
                  period, phase, meta=dict(seed=seed, name="branched"))
    w.closed = np.array(closed)
    w.parent = np.array(parent, dtype=np.int32)
    w.attach = np.array(attach, dtype=np.float64).T.copy()
    return w


# ---------------------------------------------------------------------------
# The five workloads (sizes of the paper's experiments; synthetic stand-ins).
# ---------------------------------------------------------------------------

def parity_single(seed: int = 0, nx: int = 64, ny: int = 64, n: int = 32) -> World:
    """One straight chain of ``n`` nodes along +x centred in an nx x ny box.

    Rest angles ~ N(0, 0.3^2), bond 1 cell, no actuation, fluid at rest.
    """
    g = _rng(seed)
    chain = straight_chain(n, (nx / 2.0, ny / 2.0), 0.0)
    ra = np.zeros(n)
    if n >= 3:
        ra[1:n - 1] = g.normal(0.0, 0.3, size=n - 2)
    return _assemble(nx, ny, [chain], ra, np.ones(n), [0.0], [50.0], [0.0],
                     meta=dict(seed=seed, name="single"))


def uniform_population(seed: int = 0, n_fil: int = 1024, length: int = 64, nx: int = 512,
                       ny: int = 512, amp: float = 0.5) -> World:
    """``n_fil`` chains of ``length`` nodes with sinusoidal active bending (amp rad,
    period U(20, 100) steps)."""
    w = random_world(seed, nx, ny, [length] * n_fil, amp=amp)
    w.meta["name"] = "uniform"
    return w


def scaling_lengths(seed: int, total: int, lo: int = 16, hi: int = 256) -> List[int]:
    """Lengths ~ U{lo..hi} drawn until fewer than hi + lo nodes remain; the remainder
    becomes one or two chains of length >= lo, so the lengths sum to ``total``."""
    g = _rng(seed + 7919)
    out: List[int] = []
    rem = total
    while rem >= hi + lo:
        n = int(g.integers(lo, hi + 1))
        out.append(n)
        rem -= n
    if rem > 0:
        if rem <= hi:
            out.append(rem)
        else:
            out.extend([rem // 2, rem - rem // 2])
    assert sum(out) == total and min(out) >= lo
    return out


def scaling_population(seed: int = 0, total: int = 1_048_576, nx: int = 2048, ny: int = 2048,
                       amp: float = 0.5) -> World:
    """The million-particle scaling workload: lengths U{16..256}, 2048^2 grid."""
    lengths = scaling_lengths(seed, total)
    w = random_world(seed, nx, ny, lengths, amp=amp)
    w.meta["name"] = "scaling"
    return w


def folding_population(seed: int = 0, n_fil: int = 64, length: int = 48, nx: int = 256,
                       ny: int = 256) -> World:
    """Differentiation workload: no actuation, plus a seeded smooth target fold per chain.

    Target: a chain with unit bonds whose turning angles are
    k_j = sum_{m=1..3} a_m sin(pi m (j+1)/(n-1) + b_m), a ~ N(0, 0.3^2),
    b ~ U(0, 2 pi), placed at the chain's initial centroid and orientation.
    """
    w = random_world(seed, nx, ny, [length] * n_fil, amp=0.0)
    g = _rng(seed + 104729)
    tgt = []
    for f in range(n_fil):
        a = g.normal(0.0, 0.3, size=3)
        b = g.uniform(0.0, 2.0 * math.pi, size=3)
        j = np.arange(length - 2, dtype=np.float64)
        kappa = sum(a[m] * np.sin(math.pi * (m + 1) * (j + 1) / (length - 1) + b[m]) for m in range(3))
        heading = w.meta["orient"][f] + np.concatenate([[0.0], np.cumsum(kappa)])
        pts = np.zeros((2, length))
        pts[0, 1:] = np.cumsum(np.cos(heading))
        pts[1, 1:] = np.cumsum(np.sin(heading))
        pts -= pts.mean(axis=1, keepdims=True)
        pts += w.meta["centres"][f][:, None]
        tgt.append(pts)
    w.target = np.concatenate(tgt, axis=1)
    w.meta["name"] = "folding"
    return w


def curled_chain(g: np.random.Generator, n: int, centre, turn_sd: float, bond: float = 1.0) -> np.ndarray:
    """A chain of unit bonds whose turning angles are i.i.d. N(0, turn_sd^2)
    (a persistent random walk), centroid at ``centre``: [2, n]."""
    heading = g.uniform(0.0, 2.0 * math.pi) + np.concatenate([[0.0], np.cumsum(g.normal(0.0, turn_sd, size=n - 2))])
    pts = np.zeros((2, n))
    pts[0, 1:] = np.cumsum(bond * np.cos(heading))
    pts[1, 1:] = np.cumsum(bond * np.sin(heading))
    return pts - pts.mean(axis=1, keepdims=True) + np.asarray(centre, dtype=np.float64)[:, None]


def stroke_image(g: np.random.Generator, width: int, height: int, radius: float, stroke: float) -> np.ndarray:
    """A seeded target image [height, width] in [0, 1]: a smooth closed random
    curve (radius about ``radius`` pixels around the centre, three random
    harmonics) drawn as a stroke of Gaussian profile (``stroke`` pixels)."""
    s = np.linspace(0.0, 2.0 * math.pi, 720, endpoint=False)
    r = radius * (1.0 + sum(g.normal(0.0, 0.12) * np.cos((m + 2) * s + g.uniform(0, 2 * math.pi))
                            for m in range(3)))
    px = width / 2.0 + r * np.cos(s) - 0.5
    py = height / 2.0 + r * np.sin(s) - 0.5
    a = np.arange(width, dtype=np.float64)
    b = np.arange(height, dtype=np.float64)
    d2 = np.full((height, width), np.inf)
    for x, y in zip(px, py):
        d2 = np.minimum(d2, (a[None, :] - x) ** 2 + (b[:, None] - y) ** 2)
    return np.exp(-d2 / (2.0 * stroke * stroke))


def density_folding(seed: int = 0, n: int = 1000, nx: int = 256, ny: int = 256, width: int = 128,
                    height: int = 128) -> World:
    """The paper's folding experiment at its sizes (one 1000-node filament, a
    128 x 128 loss image): a curled chain (persistent random walk, turning
    angles N(0, 0.5^2)) in the middle of a 256^2 world, rest angles
    N(0, 0.3^2), no actuation; ``meta['image']`` holds a seeded target
    image (a closed stroke, standing in for a digit image)."""
    g = _rng(seed + 15485863)
    chain = curled_chain(g, n, (nx / 2.0, ny / 2.0), 0.5)
    ra = np.zeros(n)
    ra[1:n - 1] = g.normal(0.0, 0.3, size=n - 2)
    w = _assemble(nx, ny, [chain], ra, np.ones(n), [0.0], [50.0], [0.0],
                  meta=dict(seed=seed, name="density_folding"))
    w.meta["image"] = stroke_image(g, width, height, radius=0.22 * min(width, height), stroke=1.2)
    return w


def energy_world(seed: int = 0, nx: int = 256, ny: int = 256, n_fil: int = 64, length: int = 48,
                 n_packets: int = 24, amp: float = 0.5) -> World:
    """A chemotaxis world: swimming chains (sinusoidal bending) and packets
    of energy at uniform random positions, amplitudes U(0.5, 2), widths
    U(3, 12) cells (``meta['packets']`` = (centres [2, P], amps, widths)); the
    initial field ``energy`` is left to be built from them."""
    w = random_world(seed, nx, ny, [length] * n_fil, amp=amp)
    g = _rng(seed + 49979687)
    centres = g.uniform(0.0, 1.0, size=(2, n_packets)) * np.array([[nx], [ny]])
    amps = g.uniform(0.5, 2.0, size=n_packets)
    widths = g.uniform(3.0, 12.0, size=n_packets)
    w.meta.update(name="energy", packets=(centres, amps, widths))
    return w


@dataclass
class Job:
    """One rollout job of the served workload."""

    job_id: int
    arrival: float        # seconds after trace start
    steps: int
    world: World


def served_jobs(seed: int = 0, n_jobs: int = 256, rate: float = 50.0, max_fil: int = 512,
                len_range=(8, 128), side_range=(128, 512), side_step: int = 32,
                steps_range=(200, 2000), make_world: bool = True) -> List[Job]:
    """Jobs with filament counts log-uniform on [1, max_fil], lengths U{8..128},
    grid side U{128, 160, ..., 512}, steps U{200..2000}, Poisson arrivals at ``rate``/s."""
    g = _rng(seed + 31337)
    sides = np.arange(side_range[0], side_range[1] + 1, side_step)
    jobs = []
    t = 0.0
    for j in range(n_jobs):
        t += float(g.exponential(1.0 / rate))
        n_fil = int(round(math.exp(g.uniform(0.0, math.log(max_fil)))))
        n_fil = max(1, n_fil)
        lengths = [int(v) for v in g.integers(len_range[0], len_range[1] + 1, size=n_fil)]
        side = int(g.choice(sides))
        steps = int(g.integers(steps_range[0], steps_range[1] + 1))
        wseed = int(g.integers(0, 2**31 - 1))
        w = random_world(wseed, side, side, lengths, amp=0.5) if make_world else None
        jobs.append(Job(job_id=j, arrival=t, steps=steps, world=w))
    return jobs

