"""Synthetic drift-chamber generator: geometry, determinism and event structure."""
import math

import numpy as np

from paper_2607_04067_amd import synth


def test_geometry():
    r = synth.layer_radii()
    n = synth.layer_cells()
    assert r.size == 48 and r[0] == 200.0 and abs(r[-1] - 810.0) < 1e-9
    assert n[0] == 128 and n[-1] == 384 and int(n.sum()) == synth.N_CELLS == 12288
    assert np.all(np.diff(n) > 0)


def test_deterministic_and_subset_consistent():
    a = synth.make_events("plain-16ev-180x128", 0, n_events=4)
    b = synth.make_events("plain-16ev-180x128", 0, n_events=4)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.offsets, b.offsets)
    c = synth.make_events("plain-16ev-180x128", 0, n_events=2, first=2)   # events are seeded one by one
    assert np.array_equal(c.x, a.x[a.offsets[2]:a.offsets[4]])
    d = synth.make_events("plain-16ev-180x128", 1, n_events=4)
    assert not np.array_equal(d.x, a.x)
    s = a.subset([3, 1])
    assert np.array_equal(s.event(0)[0], a.event(3)[0]) and np.array_equal(s.event(1)[1], a.event(1)[1])


def test_hits_lie_on_wires():
    ev = synth.make_events("paper-1000ev-360x256", 0, n_events=3)
    r = np.hypot(ev.x.astype(np.float64), ev.y.astype(np.float64))
    radii = synth.layer_radii()
    dist = np.abs(r[:, None] - radii[None, :]).min(axis=1)
    assert dist.max() < 1e-3


def test_plain_workload_structure():
    wl = synth.WORKLOADS["plain-16ev-180x128"]
    ev = synth.make_events(wl, 0)
    assert ev.n_events == 16 and ev.x.dtype == np.float32 and ev.offsets.dtype == np.uint32
    h = ev.hits_per_event()
    sig = np.array([int((ev.labels[ev.offsets[e]:ev.offsets[e + 1]] >= 0).sum()) for e in range(16)])
    assert np.all(sig == 3 * 48)        # 3 non-curling tracks cross all 48 layers once
    assert 300 < h.mean() < 480         # plus ~2% of 12,288 noise cells
    assert np.all(ev.track_radius > 405.0)


def test_curlers_give_duplicate_hits():
    wl = synth.WORKLOADS["paper-1000ev-360x256"]
    ev = synth.make_events(wl, 0, n_events=200)
    curl = ev.track_radius < 405.0
    assert 0.02 < curl.mean() < 0.1
    found_dup = False
    for e in np.unique(ev.track_event[curl])[:20]:
        a, b = int(ev.offsets[e]), int(ev.offsets[e + 1])
        lab = ev.labels[a:b]; xy = np.stack([ev.x[a:b], ev.y[a:b]], 1)
        for t in np.unique(lab[lab >= 0]):
            pts = xy[lab == t]
            if len(np.unique(pts, axis=0)) < len(pts):
                found_dup = True
    assert found_dup


def test_track_hits_follow_the_circle():
    """Each signal hit is the wire of a cell crossed by its circle (within half a cell)."""
    ev = synth.make_events("plain-16ev-180x128", 0, n_events=2)
    for t in range(len(ev.track_pt)):
        e = int(ev.track_event[t]); a, b = int(ev.offsets[e]), int(ev.offsets[e + 1])
        local = t - int(np.searchsorted(ev.track_event, e))
        sel = ev.labels[a:b] == local
        x, y = ev.x[a:b][sel].astype(np.float64), ev.y[a:b][sel].astype(np.float64)
        q, phi0, R = int(ev.track_charge[t]), float(ev.track_phi0[t]), float(ev.track_radius[t])
        phi_c = phi0 - q * math.pi / 2
        cx, cy = R * math.cos(phi_c), R * math.sin(phi_c)
        r = np.hypot(x, y)
        n_cells = synth.layer_cells()[np.argmin(np.abs(r[:, None] - synth.layer_radii()[None, :]), axis=1)]
        half_cell = math.pi * r / n_cells
        assert np.all(np.abs(np.hypot(x - cx, y - cy) - R) <= half_cell * 1.01)


def test_occupancy_ranges():
    ev = synth.make_events("batch-10000ev-360x256", 0, n_events=300)
    h = ev.hits_per_event()
    assert h.min() > 200 and h.max() < 3900 and h.std() > 500
    ev = synth.make_events("dense-2000ev-720x512", 0, n_events=5)
    noise = (ev.labels < 0).sum() / 5
    assert abs(noise / synth.N_CELLS - 0.30) < 0.02
