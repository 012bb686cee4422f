"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Every output is an integer (accumulator counts, peak cells and counts, keep flags), so the bar
is equality.  Small cases cover several theta tiles and ragged tails; the full-size workloads
run in the launch configuration the benchmark uses and are checked on sampled events.
"""
import math
import sys

import numpy as np
import pytest

from paper_2607_04067_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_04067_amd import hough
    hough.load()
    return hough


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _acc_np(acc, acc_type):
    a = acc.cpu().numpy()
    return a.view(np.uint16).astype(np.int32) if acc_type == "u16" else a


def _oracle_peaks(orc, acc, T):
    pj, pk, pc, n = orc.peaks(acc, T)
    return np.stack([pj, pk, pc], 1).astype(np.int64), n


def _plain_event(H, ctx, x, y, cap):
    acc = ctx.vote(_t(x), _t(y))
    peaks, npk = ctx.peaks(acc, cap)
    keep = ctx.retain(_t(x), _t(y), peaks, npk, cap)
    return acc, peaks, npk, keep


SAMPLES = [("plain-16ev-180x128", 16), ("paper-1000ev-360x256", 4), ("batch-10000ev-360x256", 4),
           ("dense-2000ev-720x512", 2), ("paper-1000ev-1000x1000", 2)]


@pytest.mark.parametrize("name,n_events", SAMPLES)
def test_plain_path_parity(H, orc, name, n_events):
    wl = synth.WORKLOADS[name]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 0, n_events=n_events)
    for T in sorted({wl.threshold, 30, 40}):
        ctx = H.Context.for_workload(wl, threshold=T)
        for e in range(n_events):
            say(f"plain {name} T={T} event={e}")
            x, y = ev.event(e)
            acc_ref = orc.vote(g, x, y)
            cap = 1 << 15
            acc, peaks, npk, keep = _plain_event(H, ctx, x, y, cap)
            assert np.array_equal(_acc_np(acc, wl.acc), acc_ref)
            ref, n_ref = _oracle_peaks(orc, acc_ref, T)
            assert int(npk.item()) == n_ref
            assert np.array_equal(H.decode_peaks(peaks, n_ref), ref)
            keep_ref = orc.retain(g, x, y, ref[:, 0], ref[:, 1], wl.rho_window)
            assert np.array_equal(keep.cpu().numpy(), keep_ref)
        ctx.close()


def test_peaks_truncation_and_retain_windows(H, orc):
    wl = synth.WORKLOADS["paper-1000ev-360x256"]
    g = orc.Grid.of(wl)
    x, y = synth.make_events(wl, 0, n_events=1).event(0)
    acc_ref = orc.vote(g, x, y)
    for W in (0, 1, 3, 17):
        ctx = H.Context.for_workload(wl, threshold=30, rho_window=W)
        acc = ctx.vote(_t(x), _t(y))
        ref, n_ref = _oracle_peaks(orc, acc_ref, 30)
        for cap in (0, 1, 5, n_ref, n_ref + 3):
            peaks, npk = ctx.peaks(acc, cap)
            assert int(npk.item()) == n_ref
            m = min(cap, n_ref)
            assert np.array_equal(H.decode_peaks(peaks, m), ref[:m])
            keep = ctx.retain(_t(x), _t(y), peaks, npk, cap)     # retains with the first cap peaks
            keep_ref = orc.retain(g, x, y, ref[:m, 0], ref[:m, 1], W)
            assert np.array_equal(keep.cpu().numpy(), keep_ref), (W, cap)
        ctx.close()


def _batch_check(H, orc, ctx, g, T, W, x, y, offsets, max_peaks):
    import torch
    xt, yt, ot = _t(x), _t(y), _t(offsets.astype(np.int64).astype(np.int32))
    peaks, npk, keep, status = ctx.run_batch(xt, yt, ot)
    torch.cuda.synchronize()
    pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, offsets, threshold=T, rho_window=W,
                                            cap=max(max_peaks, 1), n_threads=8)
    npk = npk.cpu().numpy()[:len(offsets) - 1]
    assert np.array_equal(npk.astype(np.int64), n_ref)
    assert np.array_equal(keep.cpu().numpy()[:x.size], keep_ref)
    p = peaks.cpu().numpy()
    for e in range(len(offsets) - 1):
        m = int(min(n_ref[e], max_peaks))
        if m:
            assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), e
    return status.cpu().numpy()[:len(offsets) - 1]


@pytest.mark.parametrize("name,n_events", [("plain-16ev-180x128", 16), ("paper-1000ev-360x256", 24),
                                           ("batch-10000ev-360x256", 24), ("dense-2000ev-720x512", 4),
                                           ("paper-1000ev-1000x1000", 6)])
def test_run_batch_parity(H, orc, name, n_events):
    wl = synth.WORKLOADS[name]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 0, n_events=n_events)
    for T, mp in [(wl.threshold, 20000), (wl.threshold, 100), (40, 64)]:
        say(f"batch {name} T={T} max_peaks={mp}")
        ctx = H.Context.for_workload(wl, threshold=T, max_peaks=mp)
        st = _batch_check(H, orc, ctx, g, T, wl.rho_window, ev.x, ev.y, ev.offsets, mp)
        n_ref = orc.run_batch(g, ev.x, ev.y, ev.offsets, threshold=T, rho_window=1, cap=1)[1]
        assert np.array_equal(st & H.EV_PEAKS_TRUNCATED, (n_ref > mp).astype(np.int32))
        ctx.close()


@pytest.mark.parametrize("name", ["paper-1000ev-360x256", "dense-2000ev-720x512"])
def test_run_batch_retention_windows(H, orc, name):
    """Windows below one 32-row word, at the word size and beyond it, on both tile widths."""
    wl = synth.WORKLOADS[name]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 3, n_events=6)
    for W in (0, 2, 17, 31, 32, 45, 300):
        for groups in (1, 2):
            say(f"batch windows {name} W={W} groups={groups}")
            ctx = H.Context.for_workload(wl, threshold=30, rho_window=W, max_peaks=20000)
            try:
                ctx.set_batch_plan(8, groups, 0)
            except H.HoughError:
                ctx.close()
                continue
            _batch_check(H, orc, ctx, g, 30, W, ev.x, ev.y, ev.offsets, 20000)
            ctx.close()


def _edge_events():
    """Events that exercise every special case of the path."""
    rng = np.random.default_rng(77)
    evs = []
    evs.append((np.zeros(0, np.float32), np.zeros(0, np.float32)))                    # empty
    evs.append((np.float32([350.0]), np.float32([-120.0])))                            # one hit
    x, y = synth.random_hits(300, seed=5, r_lo=150.0, r_hi=1200.0)                     # rho out of range
    evs.append((x, y))
    x, y = synth.random_hits(200, seed=6, r_lo=199.0, r_hi=201.0)                      # |rho| at the edge
    evs.append((x, y))
    ang = rng.uniform(0, 2 * np.pi, 64)
    evs.append(((200.0 * np.cos(ang)).astype(np.float32), (200.0 * np.sin(ang)).astype(np.float32)))
    x, y = synth.random_hits(120, seed=7)
    x = x.copy(); y = y.copy()
    x[:6] = [0.0, np.nan, np.inf, 1e20, -0.0, 1e-23]; y[:6] = [0.0, 1.0, 0.0, 0.0, 0.0, 0.0]
    evs.append((x, y))                                                                 # invalid hits
    x, y = synth.random_hits(40, seed=8)
    evs.append((np.tile(x, 5), np.tile(y, 5)))                                         # duplicates
    ev = synth.make_events("dense-2000ev-720x512", 3, n_events=1)
    evs.append(ev.event(0))
    return evs


@pytest.mark.parametrize("n_theta,n_rho,lo,hi", [(180, 128, -1 / 200, 1 / 200), (61, 33, -0.004, 0.006),
                                                 (62, 64, -0.005, 0.005), (63, 100, -0.0045, 0.0047),
                                                 (125, 7, -0.003, 0.004), (1, 1, -0.005, 0.005),
                                                 (200, 320, -0.006, 0.002), (124, 31, 0.0, 0.005)])
def test_edge_cases_all_entry_points(H, orc, n_theta, n_rho, lo, hi):
    g = orc.Grid(n_theta, n_rho, lo, hi)
    evs = _edge_events()
    for T in (1, 3, 9):
        ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, 1, 512)
        for i, (x, y) in enumerate(evs):
            say(f"edge grid={n_theta}x{n_rho} T={T} event={i} hits={x.size}")
            acc_ref = orc.vote(g, x, y)
            acc, peaks, npk, keep = _plain_event(H, ctx, x, y, 1 << 16)
            assert np.array_equal(acc.cpu().numpy(), acc_ref)
            ref, n_ref = _oracle_peaks(orc, acc_ref, T)
            assert int(npk.item()) == n_ref and np.array_equal(H.decode_peaks(peaks, n_ref), ref)
            assert np.array_equal(keep.cpu().numpy(), orc.retain(g, x, y, ref[:, 0], ref[:, 1], 1))
        xs = np.concatenate([e[0] for e in evs]); ys = np.concatenate([e[1] for e in evs])
        offs = np.zeros(len(evs) + 1, np.uint32); offs[1:] = np.cumsum([e[0].size for e in evs])
        st = _batch_check(H, orc, ctx, g, T, 1, xs, ys, offs, 512)
        assert st[5] & H.EV_INVALID_HITS and not (st[2] & H.EV_INVALID_HITS)
        ctx.close()


def test_u16_accumulator_and_overflow_guard(H, orc):
    import torch
    wl = synth.WORKLOADS["plain-16ev-180x128"]
    g = orc.Grid.of(wl)
    ctx = H.Context.for_workload(wl)
    x, y = synth.random_hits(65536, seed=3)
    with pytest.raises(H.HoughError) as ei:
        ctx.vote(_t(x), _t(y))
    assert ei.value.status == H.HOUGH_EOVERFLOW
    acc = ctx.vote(_t(x[:65535]), _t(y[:65535]))             # the largest event u16 accepts
    assert np.array_equal(_acc_np(acc, "u16"), orc.vote(g, x[:65535], y[:65535]))
    ctx.close()


FUSED_MAX_HITS = 32767          # largest event the fused kernel holds; larger ones spill
ITERATIVE_MAX_HITS = 32767      # largest event of the iterative finder's batch form


def test_large_events_in_batch(H, orc):
    """Events up to the fused kernel's hit limit and beyond it (the spill path, including counts
    beyond 16 bits) all equal the oracle, in one batch, plain and gathered."""
    import torch
    g = orc.Grid(360, 256, -1 / 200, 1 / 200)
    ctx = H.Context(360, 256, -1 / 200, 1 / 200, "i32", 40, 1, 4096)
    lim = FUSED_MAX_HITS
    sizes = [lim, lim + 1, 50, 70000, 0, 3]
    parts = [synth.random_hits(n, seed=1 + i, r_lo=200, r_hi=810) for i, n in enumerate(sizes)]
    xs = np.concatenate([a for a, _ in parts]).astype(np.float32)
    ys = np.concatenate([b for _, b in parts]).astype(np.float32)
    offs = np.zeros(len(sizes) + 1, np.uint32)
    offs[1:] = np.cumsum(sizes)
    say(f"large events {sizes}")
    _batch_check(H, orc, ctx, g, 40, 1, xs, ys, offs, 4096)
    # gathered, in another order, one of them twice
    ids = np.array([3, 1, 5, 1, 0], np.int64)
    koff = np.concatenate([[0], np.cumsum([sizes[i] for i in ids])[:-1]]).astype(np.int32)
    n_keep = int(sum(sizes[i] for i in ids))
    xt, yt, ot = _t(xs), _t(ys), _t(offs.astype(np.int32))
    pk, npk, keep, st = ctx.run_batch_gather(xt, yt, ot, _t(ids.astype(np.int32)), _t(koff), keep_size=n_keep)
    torch.cuda.synchronize()
    pk_ref, n_ref, keep_ref = orc.run_batch(g, xs, ys, offs, threshold=40, rho_window=1, cap=4096)
    npk, st, keep, pk = npk.cpu().numpy(), st.cpu().numpy(), keep.cpu().numpy(), pk.cpu().numpy()
    for b, e in enumerate(ids):
        assert npk[b] == n_ref[e] and st[b] == (H.EV_PEAKS_TRUNCATED if n_ref[e] > 4096 else 0), (b, e)
        m = int(min(n_ref[e], 4096))
        assert np.array_equal(H.decode_peaks(pk[b], m), pk_ref[e, :m].astype(np.int64)), (b, e)
        assert np.array_equal(keep[koff[b]:koff[b] + sizes[e]], keep_ref[offs[e]:offs[e + 1]]), (b, e)
    ctx.close()


# grids whose rho column is taller than the fused kernel's LDS tile: the per-event path votes in
# rho slabs; the batch path holds a window of the column per event (events whose hits reach
# beyond it, and every event of the split form, run through the spill path)
TALL_GRIDS = [(360, 2048, -1 / 200, 1 / 200, 10), (1000, 1500, -0.01, 0.01, 20), (97, 4099, -1 / 150, 1 / 150, 6)]


@pytest.mark.parametrize("n_theta,n_rho,lo,hi,T", TALL_GRIDS)
def test_tall_grids_equal_the_oracle(H, orc, n_theta, n_rho, lo, hi, T):
    import torch
    g = orc.Grid(n_theta, n_rho, lo, hi)
    ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, 1, 8192)
    bp = ctx.batch_plan
    assert bp["waves_per_group"] > 0 and 0 < bp["window_rows"] < n_rho   # windows of the column
    ev = synth.make_events(synth.WORKLOADS["paper-1000ev-360x256"], 5, n_events=6)
    evs = [ev.event(e) for e in range(ev.n_events)] + _edge_events()
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    off = np.zeros(len(evs) + 1, np.uint32)
    off[1:] = np.cumsum([a.size for a, _ in evs])
    say(f"tall grid {n_theta}x{n_rho}: {len(evs)} events, {x.size} hits")
    _batch_check(H, orc, ctx, g, T, 1, x, y, off, 8192)
    # the per-event path: the accumulator (slab vote), the peak list and the keep mask
    for e in range(min(3, ev.n_events)):
        xe, ye = ev.event(e)
        acc, peaks, npk, keep = _plain_event(H, ctx, xe, ye, 8192)
        torch.cuda.synchronize()
        acc_ref = orc.vote(g, xe, ye)
        assert np.array_equal(acc.cpu().numpy().astype(np.int64), acc_ref.astype(np.int64)), e
        ref, n_ref = _oracle_peaks(orc, acc_ref, T)
        assert int(npk.item()) == n_ref
        assert np.array_equal(H.decode_peaks(peaks, min(n_ref, 8192)), ref[:8192])
        assert np.array_equal(keep.cpu().numpy(), orc.retain(g, xe, ye, ref[:, 0], ref[:, 1], 1))
    # relative threshold and the split form take the same path
    xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
    E = len(evs)
    pk, npk, keep, st = ctx.run_batch(xt, yt, ot, frac=(1, 2))
    torch.cuda.synchronize()
    pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=1, cap=8192, frac=(1, 2))
    assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref)
    assert np.array_equal(keep.cpu().numpy(), keep_ref)
    sp = ctx.run_batch_split(xt, yt, ot)
    plain = ctx.run_batch(xt, yt, ot)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(sp, plain))
    # two workgroups per CU (a shorter window: more events spill) gives the same results
    try:
        ctx.set_batch_plan(8, 1, 2)
    except H.HoughError:
        pass
    else:
        say(f"tall grid {n_theta}x{n_rho} plan {ctx.batch_plan}")
        again = ctx.run_batch(xt, yt, ot)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(again, plain))
    ctx.close()


def _stacked_events(seed: int, sizes_at_least):
    """Events made of whole paper-workload events stacked until each reaches its size (tracks
    and noise, as many as fit), then one plain event and an empty one."""
    ev = synth.make_events(synth.WORKLOADS["paper-1000ev-360x256"], seed, n_events=120)
    xs, ys, sizes, e = [], [], [], 0
    for need in sizes_at_least:
        bx, by = [], []
        while sum(a.size for a in bx) < need:
            a, b = ev.event(e)
            bx.append(a)
            by.append(b)
            e += 1
        xs += bx
        ys += by
        sizes.append(sum(a.size for a in bx))
    a, b = ev.event(e)
    xs.append(a)
    ys.append(b)
    sizes += [a.size, 0]
    off = np.zeros(len(sizes) + 1, np.uint32)
    off[1:] = np.cumsum(sizes)
    return np.concatenate(xs).astype(np.float32), np.concatenate(ys).astype(np.float32), off


@pytest.mark.parametrize("n_theta,n_rho,lo,hi,T,W", [(2, 1250, -1 / 200, 1 / 200, 3, 3),
                                                     (63, 1300, -0.0048, 0.0048, 6, 1),
                                                     (125, 2100, -1 / 195, 1 / 195, 5, 2)])
def test_spill_slabs_on_narrow_periodic_grids(H, orc, n_theta, n_rho, lo, hi, T, W):
    """Theta-periodic grids taller than a tile, so every event goes through the spill path's
    slabs: with 2 columns (both halo lanes wrap onto the two owned ones), 63 (the wrapped right
    halo falls in a second group of one owned column) and 125 (three groups, the last with one
    owned column), the edge events, absolute and relative threshold (a periodic grid's rho
    range is symmetric: the wrap reverses rho)."""
    import torch
    g = orc.Grid(n_theta, n_rho, lo, hi)
    ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, W, 4096, periodic=True)
    assert ctx.batch_plan["waves_per_group"] == 0
    ev = synth.make_events(synth.WORKLOADS["paper-1000ev-360x256"], 9, n_events=4)
    evs = [ev.event(e) for e in range(ev.n_events)] + _edge_events()
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    off = np.zeros(len(evs) + 1, np.uint32)
    off[1:] = np.cumsum([a.size for a, _ in evs])
    E = len(evs)
    say(f"narrow periodic {n_theta}x{n_rho}: {E} events, {x.size} hits")
    xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
    for frac in (None, (1, 3)):
        pk, npk, keep, st = ctx.run_batch(xt, yt, ot, frac=frac)
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=W, cap=4096, periodic=True,
                                                frac=frac)
        assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref), frac
        assert np.array_equal(keep.cpu().numpy()[:x.size], keep_ref), frac
        p = pk.cpu().numpy()
        for e in range(E):
            m = int(min(n_ref[e], 4096))
            assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), (frac, e)
    ctx.close()


@pytest.mark.parametrize("periodic", [False, True])
def test_tall_grid_dedup_with_relative_threshold(H, orc, periodic):
    """Duplicate suppression and the relative threshold together on a grid taller than a tile:
    windowed tiles (plain) or the spill path's two rounds of slab votes (theta-periodic), both
    skipping the later copies the duplicate pass marked."""
    import torch
    n_theta, n_rho, lo, hi, T, W = 150, 1400, -1 / 200, 1 / 200, 4, 1
    g = orc.Grid(n_theta, n_rho, lo, hi)
    ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, W, 4096, periodic=periodic, dedup=True)
    ev = synth.make_events(synth.WORKLOADS["paper-1000ev-360x256"], 13, n_events=5)
    evs = [ev.event(e) for e in range(ev.n_events)] + _edge_events()
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    off = np.zeros(len(evs) + 1, np.uint32)
    off[1:] = np.cumsum([a.size for a, _ in evs])
    E = len(evs)
    xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
    for frac in (None, (1, 2)):
        pk, npk, keep, st = ctx.run_batch(xt, yt, ot, frac=frac)
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=W, cap=4096, periodic=periodic,
                                                dedup=True, frac=frac)
        assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref), frac
        assert np.array_equal(keep.cpu().numpy()[:x.size], keep_ref), frac
        p = pk.cpu().numpy()
        for e in range(E):
            m = int(min(n_ref[e], 4096))
            assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), (frac, e)
    ctx.close()


@pytest.mark.parametrize("periodic", [False, True])
def test_spill_slabs_of_large_events_on_a_tall_grid(H, orc, periodic):
    """The spill path's slabs in both forms and over several slabs per column: events above
    65,535 hits (32-bit counts, 480 owned rows a slab) and between 32,768 and 65,535 (packed, 992
    rows) on 130 x 1200 bins (three column groups, two or three slabs), beside a plain event and
    an empty one; plain and theta-periodic grids, absolute and relative threshold, W = 2: every
    event's peaks, count, status and keep bytes equal the oracle's."""
    import torch
    n_theta, n_rho, lo, hi, T, W, cap = 130, 1200, -1 / 200, 1 / 200, 40, 2, 8192
    g = orc.Grid(n_theta, n_rho, lo, hi)
    ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, W, cap, periodic=periodic)
    x, y, off = _stacked_events(11, [65536, 32768])
    E = off.size - 1
    say(f"spill slabs periodic={periodic}: sizes {np.diff(off).tolist()}")
    xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
    for frac in (None, (1, 2)):
        pk, npk, keep, st = ctx.run_batch(xt, yt, ot, frac=frac)
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=W, cap=cap, n_threads=8,
                                                periodic=periodic, frac=frac)
        assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref), frac
        assert np.array_equal(st.cpu().numpy()[:E], np.where(n_ref > cap, H.EV_PEAKS_TRUNCATED, 0)), frac
        assert np.array_equal(keep.cpu().numpy()[:x.size], keep_ref), frac
        p = pk.cpu().numpy()
        for e in range(E):
            m = int(min(n_ref[e], cap))
            assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), (frac, e)
    ctx.close()


@pytest.mark.parametrize("flags", ["periodic", "dedup"])
def test_tall_grid_periodic_and_dedup(H, orc, flags):
    import torch
    n_theta, n_rho, lo, hi, T = 240, 1800, -1 / 200, 1 / 200, 8
    g = orc.Grid(n_theta, n_rho, lo, hi)
    ev = synth.make_events(synth.WORKLOADS["paper-1000ev-360x256"], 6, n_events=5)
    x, y, off = ev.x, ev.y, ev.offsets
    if flags == "periodic":
        ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, 1, 8192, periodic=True)
        assert ctx.batch_plan["waves_per_group"] == 0       # no windowed form: every event spills
        pk, npk, keep, st = ctx.run_batch(_t(x), _t(y), _t(off.astype(np.int32)))
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=1, cap=8192, periodic=True)
    else:
        ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, 1, 8192, dedup=True)
        assert ctx.batch_plan["window_rows"] > 0
        pk, npk, keep, st = ctx.run_batch(_t(x), _t(y), _t(off.astype(np.int32)))
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=1, cap=8192, dedup=True)
    E = ev.n_events
    assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref)
    assert np.array_equal(keep.cpu().numpy(), keep_ref)
    p = pk.cpu().numpy()
    for e in range(E):
        m = int(min(n_ref[e], 8192))
        assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), e
    ctx.close()


def test_determinism_and_batch_independence(H):
    import torch
    wl = synth.WORKLOADS["batch-10000ev-360x256"]
    ev = synth.make_events(wl, 0, n_events=300)
    ctx = H.Context.for_workload(wl, max_peaks=8192)
    xt, yt, ot = H.to_device(ev)
    first = [t.clone() for t in ctx.run_batch(xt, yt, ot)]
    for _ in range(3):
        again = ctx.run_batch(xt, yt, ot)
        assert all(torch.equal(a, b) for a, b in zip(first, again))
    for e in (0, 137, 299):            # an event alone equals the same event inside the batch
        sub = ev.subset([e])
        xs, ys, os_ = H.to_device(sub)
        p, n, k, s = ctx.run_batch(xs, ys, os_)
        a, b = int(ev.offsets[e]), int(ev.offsets[e + 1])
        assert torch.equal(n[0], first[1][e]) and torch.equal(k, first[2][a:b])
        m = min(int(n[0]), 8192)
        assert torch.equal(p[0, :m], first[0][e, :m])
    # permuting the hits of an event permutes keep and leaves the peaks unchanged
    x, y = ev.event(5)
    perm = np.random.default_rng(0).permutation(x.size)
    offs = np.array([0, x.size], np.int32)
    p1, n1, k1, _ = ctx.run_batch(_t(x), _t(y), _t(offs))
    p2, n2, k2, _ = ctx.run_batch(_t(x[perm]), _t(y[perm]), _t(offs))
    assert torch.equal(n1, n2) and torch.equal(p1, p2)
    assert np.array_equal(k1.cpu().numpy()[perm], k2.cpu().numpy())
    ctx.close()


def _host_threads() -> int:
    import os
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


@pytest.mark.parametrize("name,periodic", [("paper-1000ev-360x256", False), ("batch-10000ev-360x256", False),
                                           ("dense-2000ev-720x512", False), ("paper-1000ev-1000x1000", False),
                                           ("paper-1000ev-1000x2000", False), ("paper-1000ev-1000x2000", True)])
def test_full_size_every_event(H, orc, name, periodic):
    """The whole workload in one launch, as the benchmark times it; every event's peak list, true
    count, status and keep bytes equal the oracle's (the oracle runs on all host cores).  The
    2000-row grid runs windowed tiles, and with the theta-periodic test the spill path
    for every event."""
    import torch
    from bench import MAX_PEAKS
    wl = synth.WORKLOADS[name]
    cap = MAX_PEAKS[name]
    ev = synth.make_events(wl, 0)
    ctx = H.Context.for_workload(wl, max_peaks=cap, periodic=periodic)
    xt, yt, ot = H.to_device(ev)
    say(f"full {name} periodic={periodic}: {ev.n_events} events, {ev.n_hits} hits, plan {ctx.batch_plan}")
    peaks, npk, keep, st = ctx.run_batch(xt, yt, ot)
    torch.cuda.synchronize()
    npk = npk.cpu().numpy().astype(np.int64)
    keep = keep.cpu().numpy()
    st = st.cpu().numpy()
    peaks = peaks.cpu().numpy()
    pk_ref, n_ref, keep_ref = orc.run_batch(wl, ev.x, ev.y, ev.offsets, cap=cap, n_threads=_host_threads(),
                                            periodic=periodic)
    assert np.array_equal(npk, n_ref)
    assert np.array_equal(st, np.where(n_ref > cap, H.EV_PEAKS_TRUNCATED, 0))
    assert np.array_equal(keep, keep_ref)
    got = peaks.reshape(ev.n_events, cap, 2).view(np.uint32)
    m = np.minimum(n_ref, cap)
    slot = np.arange(cap)[None, :] < m[:, None]
    assert np.array_equal(np.where(slot, got[:, :, 0] & 0xFFFF, 0), np.where(slot, pk_ref[:, :, 0], 0))
    assert np.array_equal(np.where(slot, got[:, :, 0] >> 16, 0), np.where(slot, pk_ref[:, :, 1], 0))
    assert np.array_equal(np.where(slot, got[:, :, 1], 0), np.where(slot, pk_ref[:, :, 2], 0))
    ctx.close()


def test_largest_grid_parity(H, orc):
    """The largest n_rho the library accepts, on the plain and the batch path."""
    import torch
    big = int(H.load().hough_max_n_rho())
    assert big >= 1000                     # the paper's 1000-bin rho axis fits
    wl = synth.WORKLOADS["paper-1000ev-1000x1000"]
    g = orc.Grid(130, big, wl.rho_min, wl.rho_max)
    ev = synth.make_events(wl, 1, n_events=3)
    ctx = H.Context(130, big, wl.rho_min, wl.rho_max, "i32", 12, 1, 20000)
    say(f"largest grid 130x{big}: plan {ctx.batch_plan}")
    _batch_check(H, orc, ctx, g, 12, 1, ev.x, ev.y, ev.offsets, 20000)
    x, y = ev.event(0)
    acc = ctx.vote(_t(x), _t(y))
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy().astype(np.int64), orc.vote(g, x, y).astype(np.int64))
    ctx.close()


def test_vote_chunks_beyond_16_bits(H, orc):
    """An event of more than 65,535 hits: the plain vote adds its 16-bit chunks into acc."""
    import torch
    g = orc.Grid(70, 96, -0.005, 0.005)
    x, y = synth.random_hits(70000, seed=9)
    ctx = H.Context(70, 96, -0.005, 0.005, "i32", 5, 1, 64)
    acc = ctx.vote(_t(x), _t(y))
    torch.cuda.synchronize()
    ref = orc.vote(g, x, y)
    assert int(ref.max()) > 0
    assert np.array_equal(acc.cpu().numpy().astype(np.int64), ref.astype(np.int64))
    ctx.close()


def test_invalid_arguments(H):
    import torch
    with pytest.raises(H.HoughError):
        H.Context(360, 256, -0.005, 0.005, "i32", 0)               # threshold < 1
    with pytest.raises(H.HoughError):
        H.Context(360, 256, 0.005, -0.005)                          # empty rho range
    with pytest.raises(H.HoughError):
        H.Context(0, 256, -0.005, 0.005)
    big = int(H.load().hough_max_n_rho())
    assert big >= 512
    with pytest.raises(H.HoughError):
        H.Context(360, big + 1, -0.005, 0.005)
    ctx = H.Context(360, big, -0.005, 0.005, "i32", 3, 1, 16)
    x, y = synth.random_hits(100, seed=1)
    acc = ctx.vote(_t(x), _t(y))
    assert int(acc.sum()) > 0
    with pytest.raises(ValueError):
        ctx.vote(torch.from_numpy(x), torch.from_numpy(y))        # host tensors are refused
    ctx.close()


def test_every_launch_plan_gives_identical_results(H):
    import torch
    for name, n in [("plain-16ev-180x128", 16), ("paper-1000ev-360x256", 40), ("dense-2000ev-720x512", 6)]:
        wl = synth.WORKLOADS[name]
        ev = synth.make_events(wl, 0, n_events=n)
        ctx = H.Context.for_workload(wl, max_peaks=16384, threshold=max(wl.threshold, 20))
        xt, yt, ot = H.to_device(ev)
        ref = [t.clone() for t in ctx.run_batch(xt, yt, ot)]
        tried = 0
        for w, gr, gpc in [(4, 1, 0), (4, 2, 0), (6, 1, 0), (6, 2, 0), (8, 1, 0), (8, 2, 0), (12, 1, 0),
                           (12, 2, 0), (16, 1, 0), (16, 2, 0), (8, 1, 1), (6, 1, 3)]:
            try:
                ctx.set_batch_plan(w, gr, gpc)
            except H.HoughError:
                continue
            tried += 1
            say(f"plan {name} waves={w} groups={gr} per_cu={gpc} -> {ctx.batch_plan}")
            out = ctx.run_batch(xt, yt, ot)
            assert all(torch.equal(a, b) for a, b in zip(ref, out)), (name, w, gr, gpc)
        assert tried >= 3
        ctx.close()


def _paper_grid_events():
    """Paper-grid workload events, then events whose hits reach beyond a 512-row window (radii
    from 150 mm: the spill path), sit inside it at its edges, or need only a few rows."""
    wl = synth.WORKLOADS["paper-1000ev-1000x1000"]
    ev = synth.make_events(wl, 9, n_events=8)
    evs = [ev.event(e) for e in range(ev.n_events)] + _edge_events()
    for seed, lo, hi in [(11, 700.0, 810.0), (12, 200.0, 200.5), (13, 450.0, 460.0)]:
        evs.append(synth.random_hits(400, seed=seed, r_lo=lo, r_hi=hi))
    # tracks plus hits at 120-190 mm: beyond any 512-row window, peaks and kept hits all the same
    xr, yr = synth.random_hits(60, seed=14, r_lo=120.0, r_hi=190.0)
    evs.insert(3, (np.concatenate([evs[0][0], xr]), np.concatenate([evs[0][1], yr])))
    evs.insert(5, synth.random_hits(500, seed=15, r_lo=120.0, r_hi=810.0))
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    off = np.zeros(len(evs) + 1, np.uint32)
    off[1:] = np.cumsum([a.size for a, _ in evs])
    return wl, x, y, off


WINDOW_PLANS = [(8, 1, 2), (4, 1, 2), (6, 1, 2), (4, 1, 3)]


def test_windowed_tile_plans_equal_the_oracle(H, orc):
    """Plans with more workgroups per CU than a whole 1000-row column allows hold a window of
    rows per event; every event (those whose rows do not fit go through the spill path) equals
    the oracle, with fixed and relative thresholds, wide retention windows and gathered."""
    import torch
    wl, x, y, off = _paper_grid_events()
    g = orc.Grid.of(wl)
    E = len(off) - 1
    xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
    seen = 0
    for W in (1, 40):
        ctx = H.Context.for_workload(wl, rho_window=W, max_peaks=8192)
        assert ctx.batch_plan["window_rows"] == 0                  # the default holds the column
        for plan in WINDOW_PLANS:
            try:
                ctx.set_batch_plan(*plan)
            except H.HoughError:
                continue
            bp = ctx.batch_plan
            say(f"windowed plan {plan} W={W} -> {bp}")
            assert bp["window_rows"] > 0 and bp["window_rows"] % 32 == 0 and bp["groups_per_cu"] == plan[2]
            seen += 1
            st = _batch_check(H, orc, ctx, g, wl.threshold, W, x, y, off, 8192)
            assert np.all((st & ~(H.EV_INVALID_HITS | H.EV_PEAKS_TRUNCATED)) == 0), st
            assert int(ctx.run_batch(xt, yt, ot)[1][3]) > 0      # the spilled event has peaks
            pk, npk, keep, st = ctx.run_batch(xt, yt, ot, frac=(1, 2))
            torch.cuda.synchronize()
            pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=wl.threshold, rho_window=W, cap=8192,
                                                    n_threads=8, frac=(1, 2))
            assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref)
            assert np.array_equal(keep.cpu().numpy(), keep_ref)
            p = pk.cpu().numpy()
            for e in range(E):
                m = int(min(n_ref[e], 8192))
                assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), e
            # gathered in reverse order, and the split form (whole column) beside it
            sizes = np.diff(off.astype(np.int64))
            ids = np.arange(E)[::-1].copy()
            koff = np.concatenate([[0], np.cumsum(sizes[ids])[:-1]]).astype(np.int32)
            plain = ctx.run_batch(xt, yt, ot)
            gk = ctx.run_batch_gather(xt, yt, ot, _t(ids.astype(np.int32)), _t(koff), keep_size=int(sizes.sum()))
            sp = ctx.run_batch_split(xt, yt, ot)
            torch.cuda.synchronize()
            assert all(torch.equal(a, b) for a, b in zip(sp, plain))
            kp, kg = plain[2].cpu().numpy(), gk[2].cpu().numpy()
            for j, e in enumerate(ids):
                assert int(gk[1][j]) == int(plain[1][e]) and int(gk[3][j]) == int(plain[3][e]), e
                assert np.array_equal(kg[koff[j]:koff[j] + sizes[e]], kp[off[e]:off[e + 1]]), e
        ctx.close()
    assert seen >= 2


def test_windowed_tile_with_duplicate_suppression(H, orc):
    import torch
    wl, x, y, off = _paper_grid_events()
    g = orc.Grid.of(wl)
    E = len(off) - 1
    ctx = H.Context.for_workload(wl, max_peaks=8192, dedup=True)
    ctx.set_batch_plan(8, 1, 2)
    assert ctx.batch_plan["window_rows"] > 0
    pk, npk, keep, st = ctx.run_batch(_t(x), _t(y), _t(off.astype(np.int32)))
    torch.cuda.synchronize()
    pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=wl.threshold, rho_window=1, cap=8192,
                                            n_threads=8, dedup=True)
    assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref)
    assert np.array_equal(keep.cpu().numpy(), keep_ref)
    p = pk.cpu().numpy()
    for e in range(E):
        m = int(min(n_ref[e], 8192))
        assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), e
    ctx.close()


@pytest.mark.parametrize("plan", [None, (8, 1, 2)])
def test_deferred_retention_with_many_peaks_and_small_buffers(H, orc, plan):
    """Low thresholds on the paper grid give tiles of more than 80 peaks among tiles of few, so
    deferred peaks are flushed before a tile that retains on its own; small peak buffers stop
    deferral once the buffer would not hold a tile's peaks.  Plain, duplicate-suppressed and
    relative-threshold runs, whole-column (16-wave) and windowed plans."""
    import torch
    wl = synth.WORKLOADS["paper-1000ev-1000x1000"]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 21, n_events=12)
    xt, yt, ot = H.to_device(ev)
    E = ev.n_events
    for T, cap, dedup, frac in [(4, 20000, False, None), (6, 150, False, None), (8, 40, True, None),
                                (20, 30, False, None), (3, 20000, False, (1, 4))]:
        ctx = H.Context(wl.n_theta, wl.n_rho, wl.rho_min, wl.rho_max, "i32", T, 1, cap, dedup=dedup)
        if plan:
            ctx.set_batch_plan(*plan)
        say(f"deferred T={T} cap={cap} dedup={dedup} frac={frac} plan={ctx.batch_plan}")
        pk, npk, keep, st = ctx.run_batch(xt, yt, ot, frac=frac) if frac else ctx.run_batch(xt, yt, ot)
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, ev.x, ev.y, ev.offsets, threshold=T, rho_window=1, cap=cap,
                                                n_threads=8, dedup=dedup, frac=frac)
        assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref)
        assert np.array_equal(keep.cpu().numpy(), keep_ref)
        p = pk.cpu().numpy()
        for e in range(E):
            m = int(min(n_ref[e], cap))
            assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), e
        assert np.array_equal((st.cpu().numpy()[:E] & H.EV_PEAKS_TRUNCATED) != 0, n_ref > cap)
        ctx.close()


def test_spill_blocks_with_many_events_left(H, orc):
    """A windowed plan whose window about half of 300 events do not fit: the spill kernel's
    workgroups take the left events from blocks all over the batch; every event equals the
    oracle, in order and gathered."""
    import torch
    wl = synth.WORKLOADS["paper-1000ev-1000x1000"]
    g = orc.Grid.of(wl)
    rng = np.random.default_rng(5)
    evs = []
    for i in range(300):
        r_lo = 150.0 if rng.random() < 0.5 else 260.0         # below 200 mm: beyond a 512-row window
        evs.append(synth.random_hits(int(rng.integers(20, 400)), seed=1000 + i, r_lo=r_lo, r_hi=810.0))
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    off = np.zeros(len(evs) + 1, np.uint32)
    off[1:] = np.cumsum([a.size for a, _ in evs])
    ctx = H.Context(wl.n_theta, wl.n_rho, wl.rho_min, wl.rho_max, "i32", 3, 1, 4096)
    ctx.set_batch_plan(8, 1, 2)
    assert ctx.batch_plan["window_rows"] == 512
    _batch_check(H, orc, ctx, g, 3, 1, x, y, off, 4096)
    sizes = np.diff(off.astype(np.int64))
    ids = rng.permutation(len(evs))
    koff = np.concatenate([[0], np.cumsum(sizes[ids])[:-1]]).astype(np.int32)
    xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
    plain = ctx.run_batch(xt, yt, ot)
    gk = ctx.run_batch_gather(xt, yt, ot, _t(ids.astype(np.int32)), _t(koff), keep_size=int(sizes.sum()))
    torch.cuda.synchronize()
    kp, kg = plain[2].cpu().numpy(), gk[2].cpu().numpy()
    for j, e in enumerate(ids):
        assert int(gk[1][j]) == int(plain[1][e]) and int(gk[3][j]) == int(plain[3][e]), e
        assert np.array_equal(kg[koff[j]:koff[j] + sizes[e]], kp[off[e]:off[e + 1]]), e
    ctx.close()


def test_windowed_plans_refused_where_no_window_helps(H):
    # a periodic grid and two column groups have no windowed form; the context keeps its plan
    wl = synth.WORKLOADS["paper-1000ev-1000x1000"]
    ctx = H.Context.for_workload(wl, periodic=True)
    before = ctx.batch_plan
    with pytest.raises(H.HoughError):
        ctx.set_batch_plan(8, 1, 2)
    with pytest.raises(H.HoughError):
        ctx.set_batch_plan(8, 2, 2)
    assert ctx.batch_plan == before
    ctx.close()


def test_autotune_keeps_results(H, tmp_path):
    import torch
    from paper_2607_04067_amd import autotune
    wl = synth.WORKLOADS["paper-1000ev-360x256"]
    ev = synth.make_events(wl, 0, n_events=64)
    ctx = H.Context.for_workload(wl, max_peaks=8192)
    xt, yt, ot = H.to_device(ev)
    ref = [t.clone() for t in ctx.run_batch(xt, yt, ot)]
    outs = [torch.zeros_like(t) for t in ref]
    cache = str(tmp_path / "plans.json")
    entry = autotune.tune(ctx, xt, yt, ot, outs, mean_hits=ev.n_hits / ev.n_events, cache=cache, reps=2)
    w, g, n = entry["plan"]
    assert ctx.batch_plan["waves_per_group"] == w and ctx.batch_plan["column_groups"] == g
    assert ctx.batch_plan["groups_per_cu"] == n
    assert all(torch.equal(a, b) for a, b in zip(ref, ctx.run_batch(xt, yt, ot)))
    again = autotune.tune(ctx, xt, yt, ot, outs, mean_hits=ev.n_hits / ev.n_events, cache=cache)
    assert again["plan"] == entry["plan"]          # served from the cache
    ctx.close()


@pytest.mark.parametrize("n_events,n_other", [(200, 50), (1000, 800)])
def test_run_batch_in_hip_graph(H, n_events, n_other):
    """Capture one hough_run_batch in a graph; every replay (with eager work in between) must
    reproduce the eager result.  With more events than workgroup slots the graph holds the
    schedule pass too, and the eager batches in between rewrite the context's schedule."""
    import torch
    wl = synth.WORKLOADS["batch-10000ev-360x256"]
    ev = synth.make_events(wl, 0, n_events=n_events)
    other = synth.make_events(wl, 5, n_events=n_other)
    ctx = H.Context.for_workload(wl, max_peaks=8192)
    xt, yt, ot = H.to_device(ev)
    xo, yo, oo = H.to_device(other)
    outs = [t for t in ctx.run_batch(xt, yt, ot)]
    torch.cuda.synchronize()
    ref = [t.clone() for t in outs]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ctx.run_batch(xt, yt, ot, *outs, stream=torch.cuda.current_stream())
    for r in range(4):
        for t in outs:
            t.zero_()
        ctx.run_batch(xo, yo, oo)                   # eager work on other data between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(ref, outs)), r
    ctx.close()


def test_largest_first_schedule_keeps_results(H, orc):
    """A batch of more events than resident workgroups is taken largest first (up to 65,536
    events, in index order beyond): every event's results equal the oracle's, and those of the
    same events gathered in index order."""
    import torch
    wl = synth.WORKLOADS["batch-10000ev-360x256"]
    g = orc.Grid.of(wl)
    pool = synth.make_events(wl, 0, n_events=400)
    rng = np.random.default_rng(5)
    xs, ys, offs = [], [], [0]
    for e in range(pool.n_events):                   # sizes from empty to whole events
        x, y = pool.event(e)
        n = int(rng.integers(0, x.size + 1)) if e % 3 else x.size
        xs.append(x[:n]); ys.append(y[:n]); offs.append(offs[-1] + n)
    x = np.concatenate(xs); y = np.concatenate(ys); offs = np.array(offs, np.uint32)
    for per_cu in (1, 0):
        say(f"largest first: 400 events, {per_cu or 'all'} workgroups per CU")
        ctx = H.Context.for_workload(wl, max_peaks=4096)
        if per_cu:
            ctx.set_batch_plan(8, 1, per_cu)
        _batch_check(H, orc, ctx, g, wl.threshold, wl.rho_window, x, y, offs, 4096)
        xt, yt, ot = _t(x), _t(y), _t(offs.astype(np.int32))
        r = ctx.run_batch(xt, yt, ot)
        ids = _t(np.arange(400, dtype=np.int32))
        gth = ctx.run_batch_gather(xt, yt, ot, ids, _t(offs[:-1].astype(np.int32)), keep_size=x.size)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(r, gth))
        ctx.close()
    # beyond 65,536 events: tiny events and a few large ones, in index order
    n_ev = 65536 + 300
    sizes = rng.integers(0, 4, n_ev)
    sizes[::997] = 600
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    x, y = synth.random_hits(int(offs[-1]), seed=9, r_lo=200, r_hi=810)
    say(f"index order: {n_ev} events, {x.size} hits")
    ctx = H.Context.for_workload(wl, max_peaks=64)
    _batch_check(H, orc, ctx, g, wl.threshold, wl.rho_window, x, y, offs, 64)
    ctx.close()


def test_gather_batches_equal_plain_batches(H):
    """A batch formed from pool indices (repeats allowed, keep at batch-local offsets) gives the
    same per-event results as a CSR batch of the same events."""
    import torch
    wl = synth.WORKLOADS["paper-1000ev-360x256"]
    pool = synth.make_events(wl, 0, n_events=40)
    ctx = H.Context.for_workload(wl, max_peaks=8192)
    xt, yt, ot = H.to_device(pool)
    ids = np.array([7, 3, 3, 39, 0, 21, 7, 12], np.int64)
    sub = pool.subset(ids)
    koff = sub.offsets[:-1].astype(np.int32)
    g = ctx.run_batch_gather(xt, yt, ot, _t(ids.astype(np.int32)), _t(koff), keep_size=sub.n_hits)
    xs, ys, os_ = H.to_device(sub)
    r = ctx.run_batch(xs, ys, os_)
    torch.cuda.synchronize()
    assert torch.equal(g[1], r[1]) and torch.equal(g[3], r[3])
    assert torch.equal(g[2][:sub.n_hits], r[2][:sub.n_hits])
    for e in range(len(ids)):
        m = min(int(r[1][e]), 8192)
        assert torch.equal(g[0][e, :m], r[0][e, :m])
    ctx.close()



def test_split_gather_batches_equal_gather_batches(H):
    """The split form over pool indices gives run_batch_gather's results, bytes outside the
    batch's keep ranges untouched, on a reused workspace."""
    import torch
    wl = synth.WORKLOADS["paper-1000ev-360x256"]
    pool = synth.make_events(wl, 0, n_events=40)
    ctx = H.Context.for_workload(wl, max_peaks=8192)
    xt, yt, ot = H.to_device(pool)
    ws = ctx.split_workspace(8)
    for ids in (np.array([7, 3, 3, 39, 0, 21, 7, 12], np.int64), np.array([5, 38], np.int64)):
        sub = pool.subset(ids)
        koff = (sub.offsets[:-1] + 5).astype(np.int32)           # a 5-byte gap before the first event
        n_keep = sub.n_hits + 9
        ref = ctx.run_batch_gather(xt, yt, ot, _t(ids.astype(np.int32)), _t(koff), keep_size=n_keep,
                                   keep=torch.full((n_keep,), 0xAB, dtype=torch.uint8, device="cuda"))
        out = ctx.run_batch_split(xt, yt, ot, ws, event_ids=_t(ids.astype(np.int32)), keep_offsets=_t(koff),
                                  keep_size=n_keep, keep=torch.full((n_keep,), 0xAB, dtype=torch.uint8, device="cuda"))
        torch.cuda.synchronize()
        say(f"split gather ids={ids.tolist()}")
        assert all(torch.equal(a, b) for a, b in zip(ref, out))
        assert int((out[2][:5] != 0xAB).sum()) == 0 and int((out[2][-4:] != 0xAB).sum()) == 0
        assert int(ws.count_nonzero()) == 0
    ctx.close()


def _serve_pools(H, n_each=48, dedup=False, resident=True, max_peaks=16384):
    from paper_2607_04067_amd import serve
    pools = []
    for name in ("paper-1000ev-360x256", "dense-2000ev-720x512"):
        wl = synth.WORKLOADS[name]
        ev = synth.make_events(wl, 7, n_events=n_each)
        ctx = H.Context.for_workload(wl, max_peaks=max_peaks, dedup=dedup)
        pools.append(serve.Pool(ctx, ev, resident=resident))
    return pools


# shape: (streams, events per batch, arena hits, arrival rate, seconds of arrivals, max_peaks)
SERVE_SHAPES = {"small": (4, 16, 40000, 2e5, 0.002, 16384),
                "bench": (8, 256, 1 << 21, 4e5, 0.003, 8192)}


@pytest.mark.parametrize("plain,small,split,dedup,resident,shape", [
    (False, 0, 0, False, True, "small"), (False, 64, 0, False, True, "small"),
    (False, 64, 4, False, True, "small"), (False, 0, 16, False, True, "small"),
    (False, 64, 8, True, True, "small"), (True, 0, 0, False, True, "small"),
    (False, 0, 0, False, False, "small"), (False, 64, 8, True, False, "small"), (True, 0, 0, False, False, "small"),
    (False, 64, 16, False, False, "bench"), (False, 64, 16, False, True, "bench")])
def test_served_results_equal_results_alone(H, plain, small, split, dedup, resident, shape):
    """Each request's n_peaks, status, keep and peak list in the served mix (continuous
    batching over several streams, events reordered largest first inside a batch, small
    batches on the 16-wave shape or in the split form or neither, duplicate suppression on
    or off, hits resident on the device or sent with each batch, up to the benchmark's shape
    of 8 streams and 256-event batches) equal the same event processed alone; requests were
    batched together and batches on different streams overlapped in time."""
    import torch
    from paper_2607_04067_amd import serve
    n_streams, max_events, arena, rate, secs, cap = SERVE_SHAPES[shape]
    pools = _serve_pools(H, dedup=dedup, resident=resident, max_peaks=cap)
    if plain:
        rate, secs = 2e4, 0.004
    trace = serve.poisson_trace(rate, secs, [p.batch.n_events for p in pools], [0.5, 0.5], seed=3)
    assert trace.size > 20
    say(f"serving {trace.size} requests: plain={plain} small={small} split={split} dedup={dedup} "
        f"resident={resident} shape={shape}")
    res, keep, peaks = serve.run(pools, trace, n_streams=n_streams, max_batch_events=max_events,
                                 max_batch_hits=arena, plain=plain, want_keep=True, want_peaks=cap,
                                 small_batch_events=small, split_batch_events=split)
    say(f"served: {serve.summarize(trace, res)}")
    off = 0
    alone = {}
    for i, (k, e) in enumerate(zip(trace["kind"], trace["event"])):
        p = pools[k]
        if (k, e) not in alone:
            sub = p.batch.subset([int(e)])
            xs, ys, os_ = H.to_device(sub)
            pk, n, kp, st = p.ctx.run_batch(xs, ys, os_)
            torch.cuda.synchronize()
            alone[(k, e)] = (int(n[0]), int(st[0]), kp.cpu().numpy()[:sub.n_hits].copy(),
                             H.decode_peaks(pk[0], min(int(n[0]), cap)))
        n, st, kp, pl = alone[(k, e)]
        assert res["n_peaks"][i] == n
        if not plain:
            assert res["status"][i] == st
        h = kp.size
        assert np.array_equal(keep[off:off + h], kp), i
        assert np.array_equal(H.decode_peaks(peaks[i], min(n, cap)), pl), i
        off += h
    assert np.all(res["done_us"] >= res["launch_us"]) and np.all(res["launch_us"] >= trace["arrival_us"])
    assert np.all(res["slot"] < n_streams)
    if not plain:
        assert res["batch_events"].max() > 1
    # two requests on different streams were in flight at the same time
    if n_streams > 1 and not plain:
        order = np.argsort(res["launch_us"], kind="stable")
        end_by_slot = {}
        overlap = False
        for j in order:
            lo, s_j = float(res["launch_us"][j]), int(res["slot"][j])
            overlap = overlap or any(end > lo for s_, end in end_by_slot.items() if s_ != s_j)
            end_by_slot[s_j] = max(end_by_slot.get(s_j, 0.0), float(res["done_us"][j]))
        assert overlap
    for p in pools:
        p.ctx.close()


# ----------------------------------------------------- the paper's iterative peak finder (plain path)
def _iter_case(H, orc, ctx, g, x, y, floor_t, frac, rt, rr, cap=4096):
    """hough_peaks_iterative on one event against the oracle (its order form, pinned against
    the step-by-step extraction on the CPU): the list in extraction order, the true count and
    the status, whatever the number of candidates."""
    import torch
    acc = ctx.vote(_t(x), _t(y))
    pk, npk, st = ctx.peaks_iterative(acc, cap, frac, rt, rr)
    torch.cuda.synchronize()
    acc_ref = orc.vote(g, x, y)
    rj, rk, rc, n_ref = orc.peaks_iterative(acc_ref, floor_t, frac, rt, rr, max(cap, 1), sorted_form=True)
    assert int(npk.item()) == n_ref
    assert int(st.item()) == (H.EV_PEAKS_TRUNCATED if n_ref > cap else 0)
    m = min(n_ref, cap)
    got = H.decode_peaks(pk, m)
    want = np.stack([rj[:m], rk[:m], rc[:m]], 1).astype(np.int64)
    assert np.array_equal(got, want), (frac, rt, rr)
    return pk, npk, n_ref


def _candidates(orc, g, x, y, floor_t, frac):
    acc = orc.vote(g, x, y)
    thr = max(floor_t, -(-int(acc.max()) * frac[0] // frac[1]))
    return int((acc >= thr).sum())


# (frac, r_theta, r_rho) per grid, the dense grid at half of the maximum among them (tens of
# thousands of candidates: the finder walks them in several LDS chunks)
ITER_SETTINGS = {
    "paper-1000ev-360x256": [((1, 2), 5, 5), ((1, 3), 2, 8), ((2, 3), 0, 0), ((0, 1), 1, 1),
                             ((1, 2), 40, 40), ((1, 4), 3, 0)],
    "dense-2000ev-720x512": [((1, 2), 5, 5), ((1, 2), 1, 1), ((2, 3), 0, 0), ((1, 2), 40, 40), ((1, 3), 3, 0)],
    "paper-1000ev-1000x1000": [((1, 2), 5, 5), ((2, 3), 0, 0), ((1, 2), 40, 40), ((2, 5), 3, 0)],
}


@pytest.mark.parametrize("name", sorted(ITER_SETTINGS))
def test_peaks_iterative_parity(H, orc, name):
    wl = synth.WORKLOADS[name]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 0, n_events=4 if name.startswith("dense") else 2)
    for floor_t in (wl.threshold, 2):
        ctx = H.Context.for_workload(wl, threshold=floor_t)
        for e in range(ev.n_events):
            x, y = ev.event(e)
            for frac, rt, rr in ITER_SETTINGS[name]:
                say(f"iterative {name} floor={floor_t} event={e} frac={frac} window=({rt},{rr}) "
                    f"candidates={_candidates(orc, g, x, y, floor_t, frac)}")
                _iter_case(H, orc, ctx, g, x, y, floor_t, frac, rt, rr)
        ctx.close()


def test_peaks_iterative_truncation_and_dense_candidates(H, orc):
    wl = synth.WORKLOADS["paper-1000ev-1000x1000"]
    g = orc.Grid.of(wl)
    x, y = synth.make_events(wl, 0, n_events=1).event(0)
    # floor 1: the first pass sees far more cells than the LDS key buffer holds, the relative
    # threshold then leaves few, which one chunk gathers
    ctx = H.Context.for_workload(wl, threshold=1)
    acc_ref = orc.vote(g, x, y)
    assert int((acc_ref >= 1).sum()) > 16384
    _, _, n = _iter_case(H, orc, ctx, g, x, y, 1, (1, 2), 4, 4)
    for cap in (0, 1, n - 1):
        _iter_case(H, orc, ctx, g, x, y, 1, (1, 2), 4, 4, cap=cap)
    # a tiny relative threshold: every non-empty cell is a candidate (hundreds of thousands),
    # many counts tie, and a small window takes tens of thousands of peaks
    say(f"dense candidates: {_candidates(orc, g, x, y, 1, (1, 1000))}")
    _iter_case(H, orc, ctx, g, x, y, 1, (1, 1000), 1, 1, cap=100000)
    _iter_case(H, orc, ctx, g, x, y, 1, (0, 1), 0, 0, cap=50)
    with pytest.raises(H.HoughError):
        ctx.peaks_iterative(ctx.vote(_t(x), _t(y)), 16, (1, 0), 1, 1)      # frac_den == 0
    with pytest.raises(H.HoughError):
        ctx.peaks_iterative(ctx.vote(_t(x), _t(y)), 16, (1, 2), -1, 1)     # negative radius
    ctx.close()


def test_peaks_iterative_bitmap_in_device_memory(H, orc):
    """A grid whose suppression bitmap does not fit LDS beside the smallest key buffer
    (1200 x 1100 cells): the bitmap lives in device memory, per event and over a batch."""
    g = orc.Grid(1200, 1100, -1 / 200, 1 / 200)
    ev = synth.make_events(synth.WORKLOADS["paper-1000ev-360x256"], 5, n_events=3)
    ctx = H.Context(1200, 1100, -1 / 200, 1 / 200, "i32", 3, 1, 20000)
    for e in range(ev.n_events):
        x, y = ev.event(e)
        for frac, rt, rr in [((1, 2), 5, 5), ((1, 8), 2, 2), ((0, 1), 1, 1)]:
            say(f"device bitmap event={e} frac={frac} candidates={_candidates(orc, g, x, y, 3, frac)}")
            _iter_case(H, orc, ctx, g, x, y, 3, frac, rt, rr, cap=20000)
    _check_batch_iterative(H, orc, ctx, g, ev.x, ev.y, ev.offsets, 3, 1, (1, 8), 2, 2, 20000)
    ctx.close()


def test_paper_pipeline_vote_iterative_peaks_retain(H, orc):
    """Plain path with the paper's peak finder: retention against its peaks matches the oracle."""
    import torch
    wl = synth.WORKLOADS["paper-1000ev-1000x1000"]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 2, n_events=3)
    ctx = H.Context.for_workload(wl, threshold=wl.threshold)
    for e in range(ev.n_events):
        x, y = ev.event(e)
        acc = ctx.vote(_t(x), _t(y))
        pk, npk, st = ctx.peaks_iterative(acc, 256, (1, 2), 5, 5)
        keep = ctx.retain(_t(x), _t(y), pk, npk, 256)
        torch.cuda.synchronize()
        rj, rk, rc, n = orc.peaks_iterative(orc.vote(g, x, y), wl.threshold, (1, 2), 5, 5, 256)
        assert int(npk.item()) == n and n >= 1
        assert np.array_equal(keep.cpu().numpy(), orc.retain(g, x, y, rj, rk, wl.rho_window))
    ctx.close()


# ------------------------------------------------------------ candidate circles and track parameters
@pytest.mark.parametrize("name,finder", [("paper-1000ev-1000x1000", "iterative"),
                                         ("paper-1000ev-360x256", "3x3"), ("dense-2000ev-720x512", "3x3")])
def test_track_params_parity(H, orc, name, finder):
    import torch
    wl = synth.WORKLOADS[name]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 4, n_events=2)
    ctx = H.Context.for_workload(wl, threshold=max(wl.threshold, 20))
    cap = 4096
    for e in range(ev.n_events):
        x, y = ev.event(e)
        xt, yt = _t(x), _t(y)
        acc = ctx.vote(xt, yt)
        if finder == "iterative":
            pk, npk, _ = ctx.peaks_iterative(acc, cap, (1, 2), 5, 5)
        else:
            pk, npk = ctx.peaks(acc, cap)
        tr = ctx.track_params(xt, yt, pk, npk, cap, 1.0)
        torch.cuda.synchronize()
        n = min(int(npk.item()), cap)
        assert n >= 1
        got = H.decode_tracks(tr, n)
        pl = H.decode_peaks(pk, n)
        ref = orc.track_params(g, x, y, pl[:, 0], pl[:, 1], wl.rho_window, 1.0)
        say(f"tracks {name} {finder} event={e} peaks={n}")
        assert np.array_equal(got["charge"], ref[:, 5].astype(np.int32))
        assert np.array_equal(got["n_hits"], ref[:, 6].astype(np.uint32))
        for i, f in enumerate(("a", "b", "radius", "pt", "phi_c")):
            np.testing.assert_allclose(got[f], ref[:, i], rtol=1e-12, atol=1e-9, err_msg=f)
    ctx.close()


# --------------------------------------------------------------------- theta-periodic adjacency
def _theta_pi_track(g, k):
    """Circle whose line lies halfway between the last column and theta = pi (both edges vote)."""
    import math
    theta = math.pi - 0.5 * math.pi / g.n_theta
    rho = g.rho_min + (k + 0.5) * (g.rho_max - g.rho_min) / g.n_rho
    radius = 1.0 / (2.0 * rho)
    radii = synth.layer_radii()
    radii = radii[radii <= 2.0 * radius * (1 - 1e-9)]
    px, py = synth.circle_points(theta, radius, radii)
    return px.astype(np.float32), py.astype(np.float32)


@pytest.mark.parametrize("n_theta,n_rho", [(360, 256), (62, 64), (63, 100), (2, 16), (125, 7), (720, 512),
                                           (100, 800), (360, 1000)])
def test_periodic_grid_plain_and_batch(H, orc, n_theta, n_rho):
    import torch
    lo, hi = -1 / 200, 1 / 200
    g = orc.Grid(n_theta, n_rho, lo, hi)
    wl = synth.WORKLOADS["paper-1000ev-360x256"]
    ev = synth.make_events(wl, 6, n_events=3)
    xs = [ev.event(e) for e in range(ev.n_events)]
    if n_theta >= 100:
        xs.append(_theta_pi_track(g, int(n_rho * 0.66)))
    x = np.concatenate([a for a, _ in xs]); y = np.concatenate([b for _, b in xs])
    offsets = np.zeros(len(xs) + 1, np.uint32)
    offsets[1:] = np.cumsum([a.size for a, _ in xs])
    for T in (3, 12):
        ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, 1, 20000, periodic=True)
        say(f"periodic grid {n_theta}x{n_rho} T={T}")
        for e, (xe, ye) in enumerate(xs):                       # plain path
            acc = ctx.vote(_t(xe), _t(ye))
            pk, npk = ctx.peaks(acc, 20000)
            torch.cuda.synchronize()
            rj, rk, rc, n = orc.peaks(orc.vote(g, xe, ye), T, periodic=True)
            assert int(npk.item()) == n, (e, T)
            assert np.array_equal(H.decode_peaks(pk, n), np.stack([rj, rk, rc], 1).astype(np.int64))
        for groups in (1, 2):                                   # fused batch path
            try:
                ctx.set_batch_plan(8, groups, 0)
            except H.HoughError:
                continue
            xt, yt, ot = _t(x), _t(y), _t(offsets.astype(np.int32))
            peaks, npk, keep, st = ctx.run_batch(xt, yt, ot)
            torch.cuda.synchronize()
            pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, offsets, threshold=T, rho_window=1, cap=20000,
                                                    n_threads=8, periodic=True)
            assert np.array_equal(npk.cpu().numpy()[:len(xs)].astype(np.int64), n_ref)
            assert np.array_equal(keep.cpu().numpy()[:x.size], keep_ref)
            p = peaks.cpu().numpy()
            for e in range(len(xs)):
                m = int(n_ref[e])
                assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), (groups, e)
        ctx.close()


def test_periodic_needs_a_symmetric_range_and_two_columns(H):
    with pytest.raises(H.HoughError):
        H.Context(360, 256, -0.004, 0.005, "i32", 3, 1, 16, periodic=True)
    with pytest.raises(H.HoughError):
        H.Context(1, 256, -0.005, 0.005, "i32", 3, 1, 16, periodic=True)
    H.Context(2, 256, -0.005, 0.005, "i32", 3, 1, 16, periodic=True).close()


# ------------------------------------------------------------ split form (one workgroup per tile)
@pytest.mark.parametrize("name,n_events", [("plain-16ev-180x128", 16), ("paper-1000ev-360x256", 24),
                                           ("dense-2000ev-720x512", 5), ("paper-1000ev-1000x1000", 4)])
def test_split_form_equals_fused_form_and_oracle(H, orc, name, n_events):
    import torch
    wl = synth.WORKLOADS[name]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 8, n_events=n_events)
    xt, yt, ot = H.to_device(ev)
    for T, mp in [(wl.threshold, 20000), (max(wl.threshold, 30), 7)]:
        ctx = H.Context.for_workload(wl, threshold=T, max_peaks=mp)
        ws = ctx.split_workspace(ev.n_events)
        ref = [t.clone() for t in ctx.run_batch(xt, yt, ot)]
        for rep in range(2):                                   # the workspace comes back zero
            out = ctx.run_batch_split(xt, yt, ot, ws)
            torch.cuda.synchronize()
            say(f"split {name} T={T} max_peaks={mp} rep={rep}")
            assert all(torch.equal(a, b) for a, b in zip(ref, out)), (name, T, mp, rep)
            assert int(ws.count_nonzero()) == 0
        pk_ref, n_ref, keep_ref = orc.run_batch(g, ev.x, ev.y, ev.offsets, threshold=T, rho_window=1,
                                                cap=max(mp, 1), n_threads=8)
        assert np.array_equal(out[1].cpu().numpy()[:ev.n_events].astype(np.int64), n_ref)
        assert np.array_equal(out[2].cpu().numpy(), keep_ref)
        ctx.close()


def test_split_form_edge_events_plans_and_periodic(H, orc):
    import torch
    evs = _edge_events()
    big = synth.random_hits(33000, seed=4)                      # beyond the batch limit
    evs = evs + [big, (np.zeros(0, np.float32), np.zeros(0, np.float32))]
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    offsets = np.zeros(len(evs) + 1, np.uint32)
    offsets[1:] = np.cumsum([a.size for a, _ in evs])
    xt, yt, ot = _t(x), _t(y), _t(offsets.astype(np.int32))
    for periodic in (False, True):
        ctx = H.Context(125, 100, -0.005, 0.005, "i32", 3, 1, 64, periodic=periodic)
        for w, gr in [(8, 1), (4, 2), (16, 1)]:
            try:
                ctx.set_batch_plan(w, gr, 0)
            except H.HoughError:
                continue
            say(f"split edges periodic={periodic} plan={w}x{gr}")
            ref = [t.clone() for t in ctx.run_batch(xt, yt, ot)]
            ws = ctx.split_workspace(len(evs))
            out = ctx.run_batch_split(xt, yt, ot, ws)
            torch.cuda.synchronize()
            assert all(torch.equal(a, b) for a, b in zip(ref, out)), (periodic, w, gr)
            assert int(ws.count_nonzero()) == 0
        ctx.close()


# ------------------------------------------------------------ duplicate suppression (HOUGH_FLAG_DEDUP)
def _dup_events():
    """Events built around repeated hits: real curler events, every hit three times (interleaved
    and in runs), one hit many times, NaN copies, -0.0 beside 0.0, and an event above the
    duplicate pass's limit."""
    rng = np.random.default_rng(31)
    evs = []
    ev = synth.make_events("paper-1000ev-360x256", 9, n_events=3)
    evs += [ev.event(e) for e in range(3)]
    x, y = synth.random_hits(400, seed=32)
    evs.append((np.tile(x, 3), np.tile(y, 3)))
    evs.append((np.repeat(x, 3), np.repeat(y, 3)))
    evs.append((np.full(50, 300.0, np.float32), np.full(50, -250.0, np.float32)))
    xs, ys = synth.random_hits(100, seed=33)
    xs = np.concatenate([xs, np.float32([np.nan, np.nan, 0.0, -0.0, 0.0])])
    ys = np.concatenate([ys, np.float32([1.0, 1.0, 350.0, 350.0, 350.0])])
    perm = rng.permutation(xs.size)
    evs.append((xs[perm], ys[perm]))
    evs.append((np.zeros(0, np.float32), np.zeros(0, np.float32)))
    evs.append((np.float32([250.0]), np.float32([400.0])))
    big_x, big_y = synth.random_hits(9000, seed=34)            # above the duplicate pass's limit
    evs.append((np.concatenate([big_x, big_x[:100]]), np.concatenate([big_y, big_y[:100]])))
    dense = synth.make_events("dense-2000ev-720x512", 9, n_events=1)
    evs.append(dense.event(0))
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    off = np.zeros(len(evs) + 1, np.uint32)
    off[1:] = np.cumsum([a.size for a, _ in evs])
    return x, y, off


@pytest.mark.parametrize("n_theta,n_rho,lo,hi,T", [(360, 256, -1 / 200, 1 / 200, 10), (180, 128, -1 / 200, 1 / 200, 8),
                                                   (720, 512, -1 / 200, 1 / 200, 12), (125, 100, -0.005, 0.005, 3),
                                                   (360, 1000, -1 / 100, 1 / 100, 20)])
def test_dedup_batch_parity_with_oracle(H, orc, n_theta, n_rho, lo, hi, T):
    import torch
    g = orc.Grid(n_theta, n_rho, lo, hi)
    x, y, off = _dup_events()
    limit = int(H.load().hough_max_dedup_hits())
    sizes = np.diff(off.astype(np.int64))
    xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
    for periodic in (False, True):
        ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, 1, 20000, periodic=periodic, dedup=True)
        say(f"dedup {n_theta}x{n_rho} T={T} periodic={periodic}")
        pk, npk, keep, st = ctx.run_batch(xt, yt, ot)
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=1, cap=20000, n_threads=8,
                                                periodic=periodic, dedup=True)
        pk_all, n_all, keep_all = orc.run_batch(g, x, y, off, threshold=T, rho_window=1, cap=20000, n_threads=8,
                                                periodic=periodic)
        big = sizes > limit
        n_want = np.where(big, n_all, n_ref)
        npk = npk.cpu().numpy()[:len(sizes)].astype(np.int64)
        assert np.array_equal(npk, n_want)
        keep_np = keep.cpu().numpy()
        p = pk.cpu().numpy()
        for e in range(len(sizes)):
            a, b = int(off[e]), int(off[e + 1])
            want_keep = keep_all[a:b] if big[e] else keep_ref[a:b]
            assert np.array_equal(keep_np[a:b], want_keep), e
            m = int(min(n_want[e], 20000))
            want = (pk_all if big[e] else pk_ref)[e, :m]
            assert np.array_equal(H.decode_peaks(p[e], m), want.astype(np.int64)), e
        stn = st.cpu().numpy()[:len(sizes)]
        assert np.array_equal((stn & H.EV_DEDUP_SKIPPED) != 0, big)
        assert int(keep_np.max()) <= 1
        # the split form and the gather form agree with the fused kernel
        ws = ctx.split_workspace(len(sizes))
        out = ctx.run_batch_split(xt, yt, ot, ws)
        torch.cuda.synchronize()
        assert torch.equal(out[1][:len(sizes)].cpu(), torch.from_numpy(npk.astype(np.int32)))
        assert torch.equal(out[3], st) and torch.equal(out[2], keep)
        ids = np.array([6, 0, 3, 3, 10], np.int64)
        koff = np.concatenate([[0], np.cumsum(sizes[ids])[:-1]]).astype(np.int32)
        gk = ctx.run_batch_gather(xt, yt, ot, _t(ids.astype(np.int32)), _t(koff), keep_size=int(sizes[ids].sum()))
        torch.cuda.synchronize()
        for j, e in enumerate(ids):
            a, b = int(off[e]), int(off[e + 1])
            assert np.array_equal(gk[2].cpu().numpy()[koff[j]:koff[j] + (b - a)], keep_np[a:b])
            assert int(gk[1][j]) == int(npk[e])
        ctx.close()


def test_dedup_workloads_equal_oracle(H, orc):
    """Real events (curlers fire the same wires on every turn) on every workload grid."""
    import torch
    for name, n in [("paper-1000ev-360x256", 24), ("dense-2000ev-720x512", 4), ("paper-1000ev-1000x1000", 4),
                    ("plain-16ev-180x128", 16)]:
        wl = synth.WORKLOADS[name]
        g = orc.Grid.of(wl)
        ev = synth.make_events(wl, 12, n_events=n)
        ctx = H.Context.for_workload(wl, max_peaks=20000, threshold=max(wl.threshold, 20), dedup=True)
        say(f"dedup workload {name}")
        xt, yt, ot = H.to_device(ev)
        pk, npk, keep, st = ctx.run_batch(xt, yt, ot)
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, ev.x, ev.y, ev.offsets, threshold=max(wl.threshold, 20),
                                                rho_window=1, cap=20000, n_threads=8, dedup=True)
        assert np.array_equal(npk.cpu().numpy()[:n].astype(np.int64), n_ref)
        assert np.array_equal(keep.cpu().numpy(), keep_ref)
        assert int(st.cpu().numpy()[:n].max()) == 0
        ctx.close()


def test_dedup_context_rejected_by_the_per_event_vote(H):
    ctx = H.Context(180, 128, -0.005, 0.005, "i32", 8, 1, 64, dedup=True)
    x, y = synth.random_hits(10, seed=1)
    with pytest.raises(H.HoughError):
        ctx.vote(_t(x), _t(y))
    ctx.close()


def test_random_configurations(H, orc):
    """Seeded random grids, ranges, thresholds, windows, capacities and options against the
    oracle: fused and split forms, bit for bit."""
    import torch
    rng = np.random.default_rng(2024)
    pool = synth.make_events("paper-1000ev-360x256", 17, n_events=6)
    ran = 0
    for case in range(20):
        n_theta = int(rng.integers(1, 420))
        n_rho = int(rng.integers(1, 1100))
        periodic = bool(rng.random() < 0.3) and n_theta >= 2
        if periodic:
            hi = float(rng.uniform(0.001, 0.008)); lo = -hi
        else:
            lo = float(rng.uniform(-0.008, 0.002)); hi = lo + float(rng.uniform(0.0005, 0.012))
        T = int(rng.integers(1, 30))
        W = int(rng.choice([0, 1, 2, 5, 31, 33]))
        cap = int(rng.choice([0, 1, 7, 300, 5000]))
        dedup = bool(rng.random() < 0.3)
        frac = [None, (1, 2), (1, 4)][int(rng.integers(0, 3))]
        evs = [pool.event(int(e)) for e in rng.integers(0, 6, 3)]
        evs.append(synth.random_hits(int(rng.integers(0, 700)), seed=case, r_lo=120.0, r_hi=900.0))
        x = np.concatenate([a for a, _ in evs]).astype(np.float32)
        y = np.concatenate([b for _, b in evs]).astype(np.float32)
        off = np.zeros(len(evs) + 1, np.uint32)
        off[1:] = np.cumsum([a.size for a, _ in evs])
        g = orc.Grid(n_theta, n_rho, lo, hi)
        try:
            ctx = H.Context(n_theta, n_rho, lo, hi, "i32", T, W, cap, periodic=periodic, dedup=dedup)
        except H.HoughError:
            continue                                   # beyond the LDS limit for n_rho
        say(f"random case {case}: {n_theta}x{n_rho} [{lo:.4f},{hi:.4f}) T={T} W={W} cap={cap} "
            f"periodic={periodic} dedup={dedup} frac={frac}")
        xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
        if frac is not None:                           # the relative threshold has no split form
            pk, npk, keep, st = ctx.run_batch(xt, yt, ot, frac=frac)
            torch.cuda.synchronize()
            pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=W, cap=max(cap, 1),
                                                    n_threads=8, periodic=periodic, dedup=dedup, frac=frac)
            assert np.array_equal(npk.cpu().numpy()[:len(evs)].astype(np.int64), n_ref), case
            assert np.array_equal(keep.cpu().numpy(), keep_ref), case
            ctx.close()
            ran += 1
            continue
        pk, npk, keep, st = (t.clone() for t in ctx.run_batch(xt, yt, ot))
        ws = ctx.split_workspace(len(evs))
        sp = ctx.run_batch_split(xt, yt, ot, ws)
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=T, rho_window=W, cap=max(cap, 1),
                                                n_threads=8, periodic=periodic, dedup=dedup)
        E = len(evs)
        assert np.array_equal(npk.cpu().numpy()[:E].astype(np.int64), n_ref), case
        assert np.array_equal(keep.cpu().numpy(), keep_ref), case
        assert np.array_equal((st.cpu().numpy()[:E] & H.EV_PEAKS_TRUNCATED) != 0, n_ref > cap), case
        p = pk.cpu().numpy()
        for e in range(E):
            m = int(min(n_ref[e], cap))
            if m:
                assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), (case, e)
        assert torch.equal(sp[1], npk) and torch.equal(sp[2], keep) and torch.equal(sp[3], st), case
        if cap:
            assert torch.equal(sp[0], pk), case
        ctx.close()
        ran += 1
    assert ran >= 15


# ------------------------------------------------------------ the paper's finder over a batch
def _check_batch_iterative(H, orc, ctx, g, x, y, off, T, W, frac, rt, rr, cap, dedup=False):
    """hough_run_batch_iterative against the oracle's batch (every event, whatever its number of
    candidates); events above the batch path's hit limit are skipped and flagged."""
    import torch
    xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
    pk, npk, keep, st = ctx.run_batch_iterative(xt, yt, ot, frac, rt, rr)
    torch.cuda.synchronize()
    E = len(off) - 1
    pk_ref, n_ref, keep_ref = orc.run_batch_iterative_fast(g, x, y, off, T, frac, rt, rr, W, cap, dedup=dedup,
                                                           n_threads=_host_threads())
    npk, st, keep, p = npk.cpu().numpy()[:E], st.cpu().numpy()[:E], keep.cpu().numpy(), pk.cpu().numpy()
    for e in range(E):
        a, b = int(off[e]), int(off[e + 1])
        if b - a > ITERATIVE_MAX_HITS:
            assert st[e] & H.EV_TOO_MANY_HITS and npk[e] == 0 and not keep[a:b].any()
            continue
        assert npk[e] == n_ref[e], e
        m = int(min(n_ref[e], cap))
        if m:
            assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), e
        assert np.array_equal(keep[a:b], keep_ref[a:b]), e
        assert bool(st[e] & H.EV_PEAKS_TRUNCATED) == (n_ref[e] > cap), e


@pytest.mark.parametrize("name,n_events,frac,rt,rr", [("paper-1000ev-360x256", 24, (1, 2), 5, 5),
                                                      ("paper-1000ev-360x256", 12, (1, 3), 2, 3),
                                                      ("dense-2000ev-720x512", 4, (1, 2), 5, 5),
                                                      ("paper-1000ev-1000x1000", 4, (1, 2), 5, 5),
                                                      ("plain-16ev-180x128", 16, (2, 3), 1, 1)])
def test_batch_iterative_parity(H, orc, name, n_events, frac, rt, rr):
    wl = synth.WORKLOADS[name]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 14, n_events=n_events)
    floor_t = max(wl.threshold, 20) if name == "paper-1000ev-1000x1000" else wl.threshold
    for cap, W, dedup in [(4096, 1, False), (3, 2, False), (4096, 1, True)]:
        say(f"batch iterative {name} frac={frac} r={rt},{rr} cap={cap} W={W} dedup={dedup}")
        ctx = H.Context.for_workload(wl, max_peaks=cap, threshold=floor_t, rho_window=W, dedup=dedup)
        _check_batch_iterative(H, orc, ctx, g, ev.x, ev.y, ev.offsets, floor_t, W, frac, rt, rr, cap, dedup)
        ctx.close()


def test_batch_iterative_edge_events_and_per_event_path(H, orc):
    """Edge events (empty, one hit, invalid hits, out of range, too many hits), a threshold so
    low that events have more candidates than one LDS chunk, and equality with the per-event
    path."""
    import torch
    evs = _edge_events() + [synth.random_hits(33000, seed=4)]
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    off = np.zeros(len(evs) + 1, np.uint32)
    off[1:] = np.cumsum([a.size for a, _ in evs])
    for T, frac in [(3, (1, 2)), (1, (0, 1))]:
        ctx = H.Context(200, 128, -0.005, 0.005, "i32", T, 1, 256)
        g = orc.Grid(200, 128, -0.005, 0.005)
        say(f"batch iterative edges T={T} frac={frac}")
        _check_batch_iterative(H, orc, ctx, g, x, y, off, T, 1, frac, 3, 3, 256)
        if frac == (0, 1):
            assert max(_candidates(orc, g, a, b, T, frac) for a, b in evs[:-1]) > 16384
        # the per-event path gives the same lists for every event that fits
        xt, yt, ot = _t(x), _t(y), _t(off.astype(np.int32))
        pk, npk, keep, st = ctx.run_batch_iterative(xt, yt, ot, frac, 3, 3)
        torch.cuda.synchronize()
        for e in range(len(evs) - 1):
            a, b = int(off[e]), int(off[e + 1])
            acc = ctx.vote(_t(x[a:b]), _t(y[a:b]))
            p1, n1, s1 = ctx.peaks_iterative(acc, 256, frac, 3, 3)
            torch.cuda.synchronize()
            assert int(n1.item()) == int(npk[e]) and int(s1.item()) == int(st[e]) & H.EV_PEAKS_TRUNCATED, e
            m = min(int(n1.item()), 256)
            assert torch.equal(p1[:m], pk[e, :m]), e
        ctx.close()


# ------------------------------------------------------------ relative threshold on the fused path
@pytest.mark.parametrize("name,n_events", [("paper-1000ev-360x256", 24), ("dense-2000ev-720x512", 4),
                                           ("paper-1000ev-1000x1000", 4), ("plain-16ev-180x128", 16)])
def test_relative_threshold_parity(H, orc, name, n_events):
    import torch
    wl = synth.WORKLOADS[name]
    g = orc.Grid.of(wl)
    ev = synth.make_events(wl, 15, n_events=n_events)
    xt, yt, ot = H.to_device(ev)
    for frac, periodic, dedup, cap in [((1, 2), False, False, 20000), ((1, 3), True, False, 20000),
                                       ((2, 3), False, True, 20000), ((1, 2), False, False, 5)]:
        say(f"relative {name} frac={frac} periodic={periodic} dedup={dedup} cap={cap}")
        ctx = H.Context.for_workload(wl, max_peaks=cap, periodic=periodic, dedup=dedup)
        pk, npk, keep, st = ctx.run_batch(xt, yt, ot, frac=frac)
        torch.cuda.synchronize()
        pk_ref, n_ref, keep_ref = orc.run_batch(g, ev.x, ev.y, ev.offsets, threshold=wl.threshold, rho_window=1,
                                                cap=cap, n_threads=8, periodic=periodic, dedup=dedup, frac=frac)
        assert np.array_equal(npk.cpu().numpy()[:n_events].astype(np.int64), n_ref)
        assert np.array_equal(keep.cpu().numpy(), keep_ref)
        p = pk.cpu().numpy()
        for e in range(n_events):
            m = int(min(n_ref[e], cap))
            assert np.array_equal(H.decode_peaks(p[e], m), pk_ref[e, :m].astype(np.int64)), e
        assert np.array_equal((st.cpu().numpy()[:n_events] & H.EV_PEAKS_TRUNCATED) != 0, n_ref > cap)
        ctx.close()


def test_relative_threshold_edge_events(H, orc):
    import torch
    evs = _edge_events() + [synth.random_hits(33000, seed=4)]
    x = np.concatenate([a for a, _ in evs]).astype(np.float32)
    y = np.concatenate([b for _, b in evs]).astype(np.float32)
    off = np.zeros(len(evs) + 1, np.uint32)
    off[1:] = np.cumsum([a.size for a, _ in evs])
    g = orc.Grid(125, 100, -0.005, 0.005)
    ctx = H.Context(125, 100, -0.005, 0.005, "i32", 2, 1, 4096)
    for frac in [(1, 2), (0, 1), (1, 1), (7, 5)]:
        pk, npk, keep, st = ctx.run_batch(_t(x), _t(y), _t(off.astype(np.int32)), frac=frac)
        torch.cuda.synchronize()
        E = len(evs)
        pk_ref, n_ref, keep_ref = orc.run_batch(g, x, y, off, threshold=2, rho_window=1, cap=4096, frac=frac)
        npk = npk.cpu().numpy()[:E]
        assert np.array_equal(npk.astype(np.int64), n_ref), frac        # the last event spills
        assert np.array_equal(st.cpu().numpy()[:E] & H.EV_TOO_MANY_HITS, np.zeros(E, np.int32))
        assert np.array_equal(keep.cpu().numpy(), keep_ref), frac
        if frac == (7, 5):
            assert npk[:E - 1].sum() == 0                  # the threshold exceeds every count
    with pytest.raises(H.HoughError):
        ctx.run_batch(_t(x), _t(y), _t(off.astype(np.int32)), frac=(1, 0))
    ctx.close()
