"""Seeded synthetic drift-chamber events (input generator shared by tests, bench and oracle checks).

This module produces hit wire positions only.  It contains none of the Hough-transform
arithmetic (no conformal map, no binning, no voting): both the HIP path and the CPU oracle
receive the arrays it returns and do all of the method's work themselves.

Detector model (a stand-in for the simulated STCF main drift chamber samples of Sec. IV,
which are not available): 48 cylindrical layers with radii linear from 200 mm to 810 mm and
cell counts linear from 128 to 384 (12,288 cells), wire at the azimuthal centre of each cell,
no stagger.  Tracks are circles through the origin in a uniform field B (Sec. II models the
transverse trajectory of a charged particle as a circular arc through the interaction point).
A track hits the wire of the cell it crosses on every layer it reaches; tracks with radius
R < 405 mm ("curlers") come back through the inner layers, and every extra turn re-fires the
same wires, producing exact duplicate hits.  Noise fires every cell independently with the
event's occupancy.  Coordinates are computed in float64 and stored as float32 (mm).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_LAYERS = 48
R_INNER_MM = 200.0
R_OUTER_MM = 810.0
CELLS_INNER = 128
CELLS_OUTER = 384
# p_T[GeV/c] = 0.299792458 * B[T] * R[m]
C_LIGHT_GEV_PER_T_M = 0.299792458


def layer_radii() -> np.ndarray:
    l = np.arange(N_LAYERS, dtype=np.float64)
    return R_INNER_MM + (R_OUTER_MM - R_INNER_MM) * l / (N_LAYERS - 1)


def layer_cells() -> np.ndarray:
    l = np.arange(N_LAYERS, dtype=np.float64)
    return np.floor(CELLS_INNER + (CELLS_OUTER - CELLS_INNER) * l / (N_LAYERS - 1) + 0.5).astype(np.int64)


_RADII = layer_radii()
_CELLS = layer_cells()
_CELL_LAYER = np.repeat(np.arange(N_LAYERS), _CELLS)                 # layer of each global cell
_CELL_INDEX = np.concatenate([np.arange(n) for n in _CELLS])         # index of the cell in its layer
_CELL_PHI = 2.0 * np.pi * (_CELL_INDEX + 0.5) / _CELLS[_CELL_LAYER]
_CELL_X = _RADII[_CELL_LAYER] * np.cos(_CELL_PHI)
_CELL_Y = _RADII[_CELL_LAYER] * np.sin(_CELL_PHI)
_LAYER_FIRST_CELL = np.concatenate([[0], np.cumsum(_CELLS)[:-1]])
N_CELLS = int(_CELLS.sum())   # 12,288


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: event mix plus the (theta, rho) grid it is processed on."""
    name: str
    n_events: int
    tracks: tuple[int, int]            # inclusive range, uniform integer
    pt_gev: tuple[float, float]        # uniform
    occupancy: tuple[float, float]     # uniform per event (lo == hi for a fixed occupancy)
    n_theta: int
    n_rho: int
    acc: str                           # "u16" or "i32": accumulator type of the plain path
    threshold: int
    rho_window: int = 1
    rho_min: float = -1.0 / 200.0      # mm^-1
    rho_max: float = 1.0 / 200.0
    b_tesla: float = 1.0
    salt: int = 0                      # separates the random streams of different workloads


WORKLOADS: dict[str, Workload] = {w.name: w for w in [
    Workload("plain-16ev-180x128", 16, (3, 3), (0.2, 1.0), (0.02, 0.02), 180, 128, "u16", 8, salt=1),
    Workload("paper-1000ev-360x256", 1000, (2, 8), (0.05, 1.5), (0.10, 0.10), 360, 256, "i32", 10, salt=2),
    Workload("batch-10000ev-360x256", 10000, (1, 12), (0.05, 1.5), (0.02, 0.25), 360, 256, "i32", 10, salt=3),
    Workload("dense-2000ev-720x512", 2000, (12, 12), (0.05, 1.5), (0.30, 0.30), 720, 512, "i32", 12, salt=4),
    # the paper's own grid (1000 x 1000 bins, rho in [-0.01, 0.01)) over the very events of the
    # 1,000-event workload (same generator and salt)
    Workload("paper-1000ev-1000x1000", 1000, (2, 8), (0.05, 1.5), (0.10, 0.10), 1000, 1000, "i32", 20,
             rho_min=-0.01, rho_max=0.01, salt=2),
    # the same events on a rho axis twice as fine (2000 rows: taller than a whole-column tile
    # on chip, so windowed tiles, and the spill path on a theta-periodic grid); a bin
    # half as tall collects fewer votes, and threshold 14 gives about the peak count (95 per
    # event) that 20 gives on the 1000-row grid (110)
    Workload("paper-1000ev-1000x2000", 1000, (2, 8), (0.05, 1.5), (0.10, 0.10), 1000, 2000, "i32", 14,
             rho_min=-0.01, rho_max=0.01, salt=2),
]}


@dataclasses.dataclass
class EventBatch:
    """CSR-packed events: hits of event e are x[offsets[e]:offsets[e+1]] (float32 SoA)."""
    x: np.ndarray          # float32 [H]
    y: np.ndarray          # float32 [H]
    offsets: np.ndarray    # uint32 [E+1]
    labels: np.ndarray     # int32 [H]: track index within the event, -1 for noise
    track_event: np.ndarray
    track_pt: np.ndarray
    track_charge: np.ndarray
    track_phi0: np.ndarray
    track_radius: np.ndarray

    @property
    def n_events(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_hits(self) -> int:
        return int(self.offsets[-1])

    def hits_per_event(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))

    def event(self, e: int) -> tuple[np.ndarray, np.ndarray]:
        a, b = int(self.offsets[e]), int(self.offsets[e + 1])
        return self.x[a:b], self.y[a:b]

    def subset(self, events) -> "EventBatch":
        events = np.asarray(events, dtype=np.int64)
        xs, ys, ls, sizes = [], [], [], []
        for e in events:
            a, b = int(self.offsets[e]), int(self.offsets[e + 1])
            xs.append(self.x[a:b]); ys.append(self.y[a:b]); ls.append(self.labels[a:b]); sizes.append(b - a)
        offsets = np.zeros(len(events) + 1, dtype=np.uint32)
        offsets[1:] = np.cumsum(sizes)
        keep = np.isin(self.track_event, events)
        remap = {int(e): i for i, e in enumerate(events)}
        cat = lambda a, dt: np.concatenate(a).astype(dt) if a else np.zeros(0, dt)
        return EventBatch(cat(xs, np.float32), cat(ys, np.float32), offsets, cat(ls, np.int32),
                          np.array([remap[int(e)] for e in self.track_event[keep]], dtype=np.int64),
                          self.track_pt[keep], self.track_charge[keep], self.track_phi0[keep],
                          self.track_radius[keep])


def track_hits(radius_mm: float, charge: int, phi0: float, n_turns: int) -> tuple[np.ndarray, np.ndarray]:
    """Wire positions (float64) fired by one circle through the origin.

    The circle's centre sits at angle phi_c = phi0 - q*pi/2 and distance R from the origin,
    so the particle leaves the origin in direction phi0.  The circle meets the layer of
    radius r (r <= 2R) at azimuth phi_c + q*arccos(r/2R) on the way out and at
    phi_c - q*arccos(r/2R) on the way back.  Each crossing fires the wire of the cell that
    contains the crossing azimuth.
    """
    phi_c = phi0 - charge * math.pi / 2.0
    reach = _RADII <= 2.0 * radius_mm
    layers = np.nonzero(reach)[0]
    if layers.size == 0:
        return np.zeros(0), np.zeros(0)
    alpha = np.arccos(np.minimum(_RADII[layers] / (2.0 * radius_mm), 1.0))
    branches = [phi_c + charge * alpha]
    curler = 2.0 * radius_mm < R_OUTER_MM
    if curler:
        branches.append(phi_c - charge * alpha)
    turns = n_turns if curler else 1
    xs, ys = [], []
    for _ in range(turns):
        for phi in branches:
            n = _CELLS[layers]
            c = np.floor(np.mod(phi, 2.0 * np.pi) * n / (2.0 * np.pi)).astype(np.int64) % n
            g = _LAYER_FIRST_CELL[layers] + c
            xs.append(_CELL_X[g]); ys.append(_CELL_Y[g])
    return np.concatenate(xs), np.concatenate(ys)


def _event_rng(seed: int, salt: int, e: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(salt), int(e)]))


def make_event(wl: Workload, seed: int, e: int):
    """One event of workload `wl`: (x64, y64, labels, tracks) before float32 rounding."""
    rng = _event_rng(seed, wl.salt, e)
    n_tracks = int(rng.integers(wl.tracks[0], wl.tracks[1] + 1))
    occ = float(rng.uniform(*wl.occupancy)) if wl.occupancy[0] != wl.occupancy[1] else wl.occupancy[0]
    xs, ys, ls, tracks = [], [], [], []
    for t in range(n_tracks):
        pt = float(rng.uniform(*wl.pt_gev))
        q = 1 if rng.random() < 0.5 else -1
        phi0 = float(rng.uniform(0.0, 2.0 * np.pi))
        n_turns = int(rng.integers(1, 4))
        radius = 1000.0 * pt / (C_LIGHT_GEV_PER_T_M * wl.b_tesla)
        tx, ty = track_hits(radius, q, phi0, n_turns)
        xs.append(tx); ys.append(ty); ls.append(np.full(tx.size, t, dtype=np.int32))
        tracks.append((pt, q, phi0, radius))
    fired = rng.random(N_CELLS) < occ
    xs.append(_CELL_X[fired]); ys.append(_CELL_Y[fired]); ls.append(np.full(int(fired.sum()), -1, np.int32))
    x = np.concatenate(xs); y = np.concatenate(ys); lab = np.concatenate(ls)
    perm = rng.permutation(x.size)
    return x[perm], y[perm], lab[perm], tracks


def make_events(wl: Workload | str, seed: int = 0, n_events: int | None = None, first: int = 0) -> EventBatch:
    """Events first .. first+n_events-1 of workload `wl` (each event has its own seeded stream)."""
    if isinstance(wl, str):
        wl = WORKLOADS[wl]
    n = wl.n_events if n_events is None else int(n_events)
    xs, ys, ls, sizes = [], [], [], []
    te, tp, tq, tf, tr = [], [], [], [], []
    for i in range(n):
        x, y, lab, tracks = make_event(wl, seed, first + i)
        xs.append(x.astype(np.float32)); ys.append(y.astype(np.float32)); ls.append(lab); sizes.append(x.size)
        for (pt, q, phi0, radius) in tracks:
            te.append(i); tp.append(pt); tq.append(q); tf.append(phi0); tr.append(radius)
    offsets = np.zeros(n + 1, dtype=np.uint32)
    offsets[1:] = np.cumsum(sizes, dtype=np.int64)
    cat = lambda a, dt: np.concatenate(a).astype(dt) if a else np.zeros(0, dt)
    return EventBatch(cat(xs, np.float32), cat(ys, np.float32), offsets, cat(ls, np.int32),
                      np.asarray(te, np.int64), np.asarray(tp, np.float64), np.asarray(tq, np.int64),
                      np.asarray(tf, np.float64), np.asarray(tr, np.float64))


def circle_points(center_angle: float, radius_mm: float, radii_mm) -> tuple[np.ndarray, np.ndarray]:
    """Points (float64) exactly on the circle through the origin with centre
    radius*(cos a, sin a), at the given distances from the origin (outgoing branch only)."""
    r = np.asarray(radii_mm, dtype=np.float64)
    alpha = np.arccos(r / (2.0 * radius_mm))
    phi = center_angle + alpha
    return r * np.cos(phi), r * np.sin(phi)


def random_hits(n: int, seed: int, r_lo: float = 150.0, r_hi: float = 900.0) -> tuple[np.ndarray, np.ndarray]:
    """Uniform random float32 hits in an annulus (for invariance and edge-case tests)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(r_lo, r_hi, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    return (r * np.cos(phi)).astype(np.float32), (r * np.sin(phi)).astype(np.float32)
