"""Benchmark of the conformal Hough hot path on one MI355X.

A step is one pass of the whole path (conformal map, theta sweep and vote, 3x3 peaks, retention
mask) over one batch of synthetic drift-chamber events already resident in HBM: one
hough_run_batch (the largest-first schedule pass and the persistent fused kernel), captured once
in a HIP graph and replayed, with the launch shape picked by the autotuner before timing.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-graph] [--no-tune]
                  [--plan W,G,C] [--no-cpu-baseline] [--no-plain] [--no-serve] ...

The default workload is the batching configuration: 10,000 events of uneven size (1-12 tracks,
noise occupancy U(2%, 25%)) on a 360 x 256 grid, threshold 10, +-1 rho bin window.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2607_04067_amd import synth  # noqa: E402

METRIC = "events/s + Gvotes/s on 1 MI355X; p50/p99 event latency, served vs plain"
DEFAULT_WORKLOAD = "batch-10000ev-360x256"
# Per-event capacity of the peak list; every event of these workloads fits (no truncation).
MAX_PEAKS = {"plain-16ev-180x128": 1024, "paper-1000ev-360x256": 8192,
             "batch-10000ev-360x256": 8192, "dense-2000ev-720x512": 16384,
             "paper-1000ev-1000x1000": 4096, "paper-1000ev-1000x2000": 4096}

# MI355X: 256 CUs, 4 SIMD16 units each, 2.4 GHz peak engine clock.
N_CU, LANES_PER_CU_CLK, CLOCK_HZ = 256, 64, 2.4e9
VALU_LANE_OPS_PER_S = N_CU * LANES_PER_CU_CLK * CLOCK_HZ          # 39.3 T 32-bit lane-ops/s
OPS_PER_VOTE = 4      # 2 FMA (rho), 1 float->int (bin), 1 index (cell address); the +1 is on the LDS
VOTE_PEAK_PER_S = VALU_LANE_OPS_PER_S / OPS_PER_VOTE              # 9.83 T votes/s
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # MI355X published vector fp32 peak
FLOPS_PER_VOTE = 4         # the two fmas of the bin, 2 flops each


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_of(text: str) -> str:
    """Source text without // comments, trailing blanks and blank lines (what compiles)."""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code:
            out.append(code)
    return "\n".join(out)


def kernel_source_id() -> str:
    """Short hash of the kernel sources' code; profile records carry the one they were taken
    with, so a change of comments alone does not retire them."""
    h = hashlib.sha256()
    for f in ("hough_kernels.hip", "hough_internal.h"):
        with open(os.path.join(ROOT, "paper_2607_04067_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def profiled_traffic(workload: str, plan):
    """HBM bytes per k_batch launch from the committed rocprofv3 counter summary of this
    workload (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a 1 GiB device copy).
    None when there is no summary, or the kernel sources or the launch plan differ from the
    ones the counters were taken with."""
    path = os.path.join(ROOT, "profiles", f"k_batch_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    start = text.find("```json")
    if start < 0:
        return None
    rec = json.loads(text[start + 7:text.index("```", start + 7)])
    cur = [plan["waves_per_group"], plan["column_groups"], plan["groups_per_cu"]]
    if (rec.get("source") != kernel_source_id() or rec.get("plan") != cur
            or rec.get("window_rows", 0) != plan.get("window_rows", 0)):
        return None
    return rec


def lds_atomic_ceiling(reps: int = 3) -> dict:
    """The LDS atomic rate of the vote's access pattern over the whole chip, measured here and now
    with libhough_probe.so (ds_add_u32, lane l on dword 32 * row + (l & 31), 16-bit halves, rows
    changing every instruction, nothing else in the loop): lane-updates per second, the best of
    a few occupancies, each the median of `reps` launches timed with HIP events."""
    import ctypes
    import torch
    L = ctypes.CDLL(os.path.join(ROOT, "paper_2607_04067_amd", "libhough_probe.so"))
    L.hough_probe_lds_add.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.hough_probe_lds_add.restype = ctypes.c_int
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    stream = torch.cuda.current_stream()
    rows = []
    for waves, per_cu in ((8, 3), (8, 4), (16, 2), (4, 8)):
        blocks, iters = n_cu * per_cu, 4096
        sink = torch.zeros(blocks, dtype=torch.int32, device="cuda")
        if L.hough_probe_lds_add(blocks, waves, iters, sink.data_ptr(), stream.cuda_stream) != 0:
            raise RuntimeError("hough_probe_lds_add failed")
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            L.hough_probe_lds_add(blocks, waves, iters, sink.data_ptr(), stream.cuda_stream)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        lanes = blocks * waves * 64 * iters * 8
        rows.append({"waves_per_group": waves, "groups_per_cu": per_cu, "ms": round(ms, 4),
                     "lane_updates_per_s": lanes / (ms / 1e3)})
    best = max(rows, key=lambda r: r["lane_updates_per_s"])
    return {"lane_updates_per_s": best["lane_updates_per_s"],
            "lanes_per_clk_per_cu": round(best["lane_updates_per_s"] / (n_cu * CLOCK_HZ), 2),
            "probe": "libhough_probe.so ds_add_u32 loop, best of " + ", ".join(
                f"{r['waves_per_group']}x{r['groups_per_cu']}: {r['lane_updates_per_s'] / 1e12:.2f} T/s" for r in rows)}


def lds_atomic_rate(ev, plan, wl, kern_ms: float, ceiling_per_s: float) -> dict:
    """LDS vote atomics the fused kernel issues per launch (each valid hit updates every lane's
    column of every theta tile, halo and out-of-grid lanes included: 64 * column_groups lanes per
    tile) per second of kernel time, against the measured LDS atomic ceiling."""
    x64, y64 = ev.x.astype(np.float32), ev.y.astype(np.float32)
    r2 = x64 * x64 + y64 * y64
    valid = int(np.count_nonzero((r2 > 0) & np.isfinite(r2)))
    lanes_per_tile = 64 * plan["column_groups"]
    tiles = -(-wl.n_theta // (lanes_per_tile - 2))
    lanes = valid * tiles * lanes_per_tile
    rate = lanes / (kern_ms / 1e3)
    return {"lane_updates_per_launch": lanes, "achieved_per_s": round(rate / 1e12, 3), "unit": "T/s",
            "ceiling_per_s": round(ceiling_per_s / 1e12, 3),
            "frac": round(rate / ceiling_per_s, 4)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, ev, budget_s: float = 20.0, runs: int = 10):
    """The CPU oracle, as it stands, on the host cores: a bounded sample of the workload (the
    first n events, n sized so that the `runs` timed runs cost about budget_s of CPU time in
    all), run `runs` times with OpenMP over events on up to 16 threads (the machine's CPU share for
    one GPU) and reported as the median, then once on one core."""
    from oracle import oracle
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(16, avail))
    cap = MAX_PEAKS[wl.name]
    # one-thread probe of the per-event cost
    probe = ev.subset(np.arange(min(16, ev.n_events)))
    t0 = time.perf_counter()
    oracle.run_batch(wl, probe.x, probe.y, probe.offsets, cap=cap, n_threads=1)
    per_event = (time.perf_counter() - t0) / probe.n_events
    n = int(min(ev.n_events, max(threads, budget_s / runs / max(per_event, 1e-6))))
    sample = ev.subset(np.arange(n))
    oracle.run_batch(wl, sample.x, sample.y, sample.offsets, cap=cap, n_threads=threads)   # warm-up
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.run_batch(wl, sample.x, sample.y, sample.offsets, cap=cap, n_threads=threads)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    votes = sample.n_hits * wl.n_theta
    t0 = time.perf_counter()
    oracle.run_batch(wl, sample.x, sample.y, sample.offsets, cap=cap, n_threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": round(n / dt, 2), "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of {ev.n_events} events of {wl.name} (whole path, all peaks), "
                      f"median of {runs} runs after one warm-up",
            "cpu": cpu_model(), "host_cpus": avail,
            "gvotes_per_s": round(votes / dt / 1e9, 4), "seconds": round(dt, 4),
            "one_core": {"events_per_s": round(n / dt1, 2), "sample_events": n, "seconds": round(dt1, 3),
                         "gvotes_per_s": round(votes / dt1 / 1e9, 4)}}


def plain_path(H, wl, ev, n_events: int = 200):
    """Per-event launches (vote, peaks, retain) with the accumulator in HBM, for comparison."""
    import torch
    ctx = H.Context.for_workload(wl)
    sub = ev.subset(np.arange(min(n_events, ev.n_events)))
    xt, yt, _ = H.to_device(sub)
    cap = MAX_PEAKS[wl.name]
    dt_acc = torch.int16 if wl.acc == "u16" else torch.int32
    acc = torch.empty((wl.n_theta, wl.n_rho), dtype=dt_acc, device="cuda")
    peaks = torch.zeros((cap, 2), dtype=torch.int32, device="cuda")
    npk = torch.zeros(1, dtype=torch.int32, device="cuda")
    keep = torch.zeros(sub.n_hits, dtype=torch.uint8, device="cuda")
    offs = sub.offsets.astype(np.int64)

    def one_pass():
        for e in range(sub.n_events):
            a, b = int(offs[e]), int(offs[e + 1])
            ctx.vote(xt[a:b], yt[a:b], acc)
            ctx.peaks(acc, cap, peaks, npk)
            ctx.retain(xt[a:b], yt[a:b], peaks, npk, cap, keep[a:b])

    one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # votes that land in the grid (the accumulator total), beside the attempted votes
    landed = torch.zeros((), dtype=torch.int64, device="cuda")
    for e in range(sub.n_events):
        a, b = int(offs[e]), int(offs[e + 1])
        ctx.vote(xt[a:b], yt[a:b], acc)
        cells = acc.to(torch.int64) & 0xFFFF if wl.acc == "u16" else acc.to(torch.int64)
        landed += cells.sum()
    landed_frac = float(landed.item()) / max(1, sub.n_hits * wl.n_theta)
    ctx.close()
    return {"events_per_s": round(sub.n_events / dt, 1), "events": sub.n_events,
            "launches_per_event": 3, "ms_per_event": round(dt / sub.n_events * 1e3, 4),
            "landed_vote_fraction": round(landed_frac, 5)}


def flagged(H, status) -> int:
    """Events with a status bit other than the peak buffer's truncation (which depends only on
    the buffer the caller gives): invalid hits, refusals, skipped duplicate passes."""
    return int(((np.asarray(status) & ~H.EV_PEAKS_TRUNCATED) != 0).sum())


def truncated(H, status) -> int:
    """Events with more peaks than the peak buffer holds (their counts are still the true ones)."""
    return int(((np.asarray(status) & H.EV_PEAKS_TRUNCATED) != 0).sum())


def iterative_path(H, wl, ev, n_events: int = 200, frac=(1, 2), r_theta: int = 5, r_rho: int = 5):
    """The paper's own peak finder on the per-event path: vote (accumulator in HBM), relative
    threshold + iterative extraction, retention against those peaks; three launches per event."""
    import torch
    ctx = H.Context.for_workload(wl)
    sub = ev.subset(np.arange(min(n_events, ev.n_events)))
    xt, yt, _ = H.to_device(sub)
    cap = MAX_PEAKS[wl.name]        # the batch path's peak buffer: truncation is the caller's choice
    dt_acc = torch.int16 if wl.acc == "u16" else torch.int32
    acc = torch.empty((wl.n_theta, wl.n_rho), dtype=dt_acc, device="cuda")
    peaks = torch.zeros((sub.n_events, cap, 2), dtype=torch.int32, device="cuda")
    npk = torch.zeros((sub.n_events, 1), dtype=torch.int32, device="cuda")
    st = torch.zeros((sub.n_events, 1), dtype=torch.int32, device="cuda")
    keep = torch.zeros(sub.n_hits, dtype=torch.uint8, device="cuda")
    offs = sub.offsets.astype(np.int64)

    def one_pass():
        for e in range(sub.n_events):
            a, b = int(offs[e]), int(offs[e + 1])
            ctx.vote(xt[a:b], yt[a:b], acc)
            ctx.peaks_iterative(acc, cap, frac, r_theta, r_rho, peaks[e], npk[e], st[e])
            ctx.retain(xt[a:b], yt[a:b], peaks[e], npk[e], cap, keep[a:b])

    one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    k = keep.cpu().numpy()
    lab = sub.labels
    out = {"finder": f"relative threshold {frac[0]}/{frac[1]} of the maximum (floor {wl.threshold}), "
                     f"suppression window +-{r_theta} theta x +-{r_rho} rho bins",
           "events": sub.n_events, "ms_per_event": round(dt / sub.n_events * 1e3, 4),
           "events_per_s": round(sub.n_events / dt, 1),
           "peaks_per_event": round(float(npk.float().mean().item()), 2),
           "flagged": flagged(H, st.cpu().numpy()), "truncated": truncated(H, st.cpu().numpy()),
           "peak_buffer": cap,
           "R_c": round(float(k.mean()), 4) if k.size else None,
           "R_s": round(float(k[lab >= 0].mean()), 4) if (lab >= 0).any() else None}

    # the same finder over the whole batch at once (hough_run_batch_iterative: four launches)
    bctx = H.Context.for_workload(wl, max_peaks=cap)
    bx, by, bo = H.to_device(ev)
    ws = bctx.iterative_workspace(ev.n_events)
    res = bctx.run_batch_iterative(bx, by, bo, frac, r_theta, r_rho, ws)
    times = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        bctx.run_batch_iterative(bx, by, bo, frac, r_theta, r_rho, ws, *res)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    kb = res[2].cpu().numpy()
    out["batch"] = {"events": ev.n_events, "ms": round(ms, 4), "events_per_s": round(ev.n_events / (ms / 1e3), 1),
                    "workspace_bytes": int(ws.numel()),
                    "flagged": flagged(H, res[3].cpu().numpy()[:ev.n_events]),
                    "truncated": truncated(H, res[3].cpu().numpy()[:ev.n_events]),
                    "R_c": round(float(kb.mean()), 4) if kb.size else None,
                    "R_s": round(float(kb[ev.labels >= 0].mean()), 4) if (ev.labels >= 0).any() else None}
    bctx.close()
    return out


PT_BINS = (0.05, 0.2, 0.5, 1.0, 1.5)


def physics(H, wl, ev, n_events: int = 200, frac=(1, 2), r_theta: int = 5, r_rho: int = 5):
    """Track finding against the generator's truth, with the paper's peak finder on the GPU
    (vote, relative threshold + iterative extraction, candidate circles).  A truth track's
    candidate is the peak that keeps the most of its hits (retention with that peak alone, on
    the GPU); the track counts as found when |pT_reco - pT_truth| < 20 MeV/c or that peak keeps
    more than 90% of its hits (the paper's composite criterion).  Reports the efficiency per
    pT range, and for found tracks the charge agreement and robust widths (1.4826 x median
    absolute deviation) of the phi0 residual and of the relative pT residual."""
    import torch
    ctx = H.Context.for_workload(wl)
    sub = ev.subset(np.arange(min(n_events, ev.n_events)))
    xt, yt, _ = H.to_device(sub)
    cap = 256
    acc = torch.empty((wl.n_theta, wl.n_rho), dtype=torch.int16 if wl.acc == "u16" else torch.int32,
                      device="cuda")
    offs = sub.offsets.astype(np.int64)
    one = torch.ones(1, dtype=torch.int32, device="cuda")
    found, pts, dphi, dpt, qok = [], [], [], [], []
    for e in range(sub.n_events):
        a, b = int(offs[e]), int(offs[e + 1])
        x, y = xt[a:b], yt[a:b]
        ctx.vote(x, y, acc)
        pk, npk, _ = ctx.peaks_iterative(acc, cap, frac, r_theta, r_rho)
        tr = ctx.track_params(x, y, pk, npk, cap, wl.b_tesla)
        n = min(int(npk.item()), cap)
        tracks = H.decode_tracks(tr, n)
        keeps = torch.zeros((max(n, 1), b - a), dtype=torch.uint8, device="cuda")
        for p in range(n):
            ctx.retain(x, y, pk[p:p + 1], one, 1, keeps[p])
        kp = keeps[:n].cpu().numpy().astype(bool)
        lab = sub.labels[a:b]
        for t in np.nonzero(sub.track_event == e)[0]:
            mine = lab == (t - np.searchsorted(sub.track_event, e))
            pt_true = float(sub.track_pt[t])
            pts.append(pt_true)
            if n == 0 or not mine.any():
                found.append(False)
                continue
            srr = kp[:, mine].sum(axis=1) / mine.sum()
            best = int(np.argmax(srr))
            pt_reco = float(tracks["pt"][best])
            ok = abs(pt_reco - pt_true) < 0.020 or srr[best] > 0.9
            found.append(ok)
            if ok:
                q = int(tracks["charge"][best])
                qok.append(q == int(sub.track_charge[t]))
                phi0 = float(tracks["phi_c"][best]) + q * np.pi / 2
                dphi.append(float(np.remainder(phi0 - sub.track_phi0[t] + np.pi, 2 * np.pi) - np.pi))
                dpt.append((pt_reco - pt_true) / pt_true)
    ctx.close()
    found, pts = np.array(found), np.array(pts)
    robust = lambda v: round(float(1.4826 * np.median(np.abs(np.array(v) - np.median(v)))), 5) if v else None
    by_pt = {}
    for lo, hi in zip(PT_BINS[:-1], PT_BINS[1:]):
        sel = (pts >= lo) & (pts < hi)
        by_pt[f"{lo}-{hi}"] = round(float(found[sel].mean()), 4) if sel.any() else None
    return {"events": sub.n_events, "tracks": int(found.size),
            "finder": f"relative threshold {frac[0]}/{frac[1]}, window +-{r_theta} x +-{r_rho}",
            "efficiency": round(float(found.mean()), 4) if found.size else None,
            "efficiency_by_pt_gev": by_pt,
            "charge_correct": round(float(np.mean(qok)), 4) if qok else None,
            "phi0_width_rad": robust(dphi), "pt_rel_width": robust(dpt),
            "criterion": "|pT_reco - pT_truth| < 20 MeV/c or > 90% of the track's hits kept by its peak"}


def relative_threshold(H, ctx, xt, yt, ot, peaks, npk, keep, status, ev, stream, frac=(1, 2), reps: int = 10):
    """The fused path with each event's threshold max(T, ceil(max * frac)) (the form of the
    paper's own threshold): kernel time (HIP events, median) and the resulting mask."""
    import torch
    ctx.run_batch(xt, yt, ot, peaks, npk, keep, status, stream, frac=frac)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.run_batch(xt, yt, ot, peaks, npk, keep, status, stream, frac=frac)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    k = keep.cpu().numpy()
    lab = ev.labels
    return {"frac": f"{frac[0]}/{frac[1]}", "kernel_ms": round(ms, 4),
            "events_per_s": round(ev.n_events / (ms / 1e3), 1),
            "peaks_per_event": round(float(npk.float().mean().item()), 2),
            "R_c": round(float(k.mean()), 4) if k.size else None,
            "R_s": round(float(k[lab >= 0].mean()), 4) if (lab >= 0).any() else None}


SECONDARY_WORKLOADS = ["plain-16ev-180x128", "paper-1000ev-360x256", "dense-2000ev-720x512",
                       "paper-1000ev-1000x1000"]


def secondary(H, names, ceiling: dict, tune: bool, reps: int = 20) -> dict:
    """The other configurations beside the headline, each on its own resident batch: the
    launch shape autotuned on it (or the library default), then `reps` launches of
    hough_run_batch timed with HIP events on the launch stream (mean), the LDS-atomic and
    published-fp32 fractions as in the headline's roofline, and the profiled HBM traffic where
    a summary for that workload and shape exists."""
    import torch
    lds_peak = ceiling["lane_updates_per_s"] / 1e9
    out = {}
    for name in names:
        wl = synth.WORKLOADS[name]
        ev = synth.make_events(wl, 0)
        cap = MAX_PEAKS[name]
        ctx = H.Context.for_workload(wl, max_peaks=cap)
        xt, yt, ot = H.to_device(ev)
        bufs = ctx.run_batch(xt, yt, ot)
        if tune:
            from paper_2607_04067_amd import autotune
            autotune.tune(ctx, xt, yt, ot, bufs, mean_hits=ev.n_hits / max(ev.n_events, 1), cache=None)
        stream = torch.cuda.current_stream()
        for _ in range(3):
            ctx.run_batch(xt, yt, ot, *bufs, stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            ctx.run_batch(xt, yt, ot, *bufs, stream=stream)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        plan = ctx.batch_plan
        gv = ev.n_hits * wl.n_theta / (ms / 1e3) / 1e9
        prof = profiled_traffic(name, plan)
        out[name] = {"events": ev.n_events, "hits": ev.n_hits, "plan": plan,
                     "plan_source": "autotuned" if tune else "library default",
                     "kernel_ms": round(ms, 4), "events_per_s": round(ev.n_events / (ms / 1e3), 1),
                     "gvotes_per_s": round(gv, 1), "frac": round(gv / lds_peak, 4),
                     "lds_atomic_frac": lds_atomic_rate(ev, plan, wl, ms, ceiling["lane_updates_per_s"])["frac"],
                     "fp32_frac": round(gv * 1e9 * FLOPS_PER_VOTE / 1e12 / FP32_PEAK_TFLOPS, 4),
                     "traffic": prof["traffic_bytes"] if prof else None,
                     "peaks_per_event": round(float(bufs[1].float().mean().item()), 1)}
        log(f"secondary {name}: {out[name]['kernel_ms']} ms, plan {plan}")
        ctx.close()
        del xt, yt, ot, bufs
    return out


def periodic_grid(H, wl, ev, xt, yt, ot, stream, reps: int = 10):
    """The fused path on the same grid with the theta-periodic 3x3 test (HOUGH_FLAG_THETA_PERIODIC):
    kernel time (HIP events, median), peaks and mask."""
    import torch
    ctx = H.Context.for_workload(wl, max_peaks=MAX_PEAKS[wl.name], periodic=True)
    outs = ctx.run_batch(xt, yt, ot, stream=stream)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.run_batch(xt, yt, ot, *outs, stream=stream)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    npk, k = outs[1], outs[2].cpu().numpy()
    lab = ev.labels
    out = {"kernel_ms": round(ms, 4), "events_per_s": round(ev.n_events / (ms / 1e3), 1),
           "peaks_per_event": round(float(npk.float().mean().item()), 2),
           "R_c": round(float(k.mean()), 4) if k.size else None,
           "R_s": round(float(k[lab >= 0].mean()), 4) if (lab >= 0).any() else None,
           "plan": ctx.batch_plan}
    ctx.close()
    return out


def end_to_end(H, ctx, wl, ev, reps: int = 10):
    """PCIe-inclusive rate of the batch path: hits and offsets from pinned host memory to HBM,
    one fused launch, then n_peaks, status and keep (and, in the second figure, the whole
    fixed-capacity peak buffer) back to pinned host memory, all on one stream.  Median of reps."""
    import torch
    E, cap = ev.n_events, MAX_PEAKS[wl.name]
    hx = torch.from_numpy(ev.x).pin_memory()
    hy = torch.from_numpy(ev.y).pin_memory()
    ho = torch.from_numpy(ev.offsets.astype(np.int32)).pin_memory()
    dx, dy = torch.empty_like(hx, device="cuda"), torch.empty_like(hy, device="cuda")
    do = torch.empty_like(ho, device="cuda")
    peaks = torch.zeros((E, cap, 2), dtype=torch.int32, device="cuda")
    npk = torch.zeros(E, dtype=torch.int32, device="cuda")
    keep = torch.zeros(ev.n_hits, dtype=torch.uint8, device="cuda")
    status = torch.zeros(E, dtype=torch.int32, device="cuda")
    h_npk = torch.empty(E, dtype=torch.int32).pin_memory()
    h_status = torch.empty(E, dtype=torch.int32).pin_memory()
    h_keep = torch.empty(ev.n_hits, dtype=torch.uint8).pin_memory()
    h_peaks = torch.empty((E, cap, 2), dtype=torch.int32).pin_memory()
    stream = torch.cuda.current_stream()

    def once(with_peaks):
        dx.copy_(hx, non_blocking=True)
        dy.copy_(hy, non_blocking=True)
        do.copy_(ho, non_blocking=True)
        ctx.run_batch(dx, dy, do, peaks, npk, keep, status, stream)
        h_npk.copy_(npk, non_blocking=True)
        h_status.copy_(status, non_blocking=True)
        h_keep.copy_(keep, non_blocking=True)
        if with_peaks:
            h_peaks.copy_(peaks, non_blocking=True)

    out = {"h2d_bytes": 8 * ev.n_hits + 4 * (E + 1)}
    for key, with_peaks in (("counts_keep", False), ("with_peak_buffer", True)):
        once(with_peaks)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            once(with_peaks)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        out[key] = {"ms": round(ms, 4), "events_per_s": round(E / (ms / 1e3), 1)}
    out["with_peak_buffer"]["d2h_peak_bytes"] = E * cap * 8

    return out


SERVE_RATES = (50_000, 100_000, 200_000, 400_000)


def _stage_times(H, ctx, sub, cap, reps):
    """Mean times (ms) of one batch's stages on one stream: hits and offsets from pinned host
    memory to HBM, the fused launch, n_peaks/status/keep back to pinned host memory, and the
    three together.  Each stage is bracketed by its own HIP events; the mean of reps runs."""
    import torch
    E = sub.n_events
    hx = torch.from_numpy(np.ascontiguousarray(sub.x)).pin_memory()
    hy = torch.from_numpy(np.ascontiguousarray(sub.y)).pin_memory()
    ho = torch.from_numpy(sub.offsets.astype(np.int32)).pin_memory()
    dx, dy, do = (torch.empty_like(t, device="cuda") for t in (hx, hy, ho))
    peaks = torch.zeros((E, cap, 2), dtype=torch.int32, device="cuda")
    npk = torch.zeros(E, dtype=torch.int32, device="cuda")
    keep = torch.zeros(max(sub.n_hits, 1), dtype=torch.uint8, device="cuda")
    status = torch.zeros(E, dtype=torch.int32, device="cuda")
    h_npk, h_st = torch.empty(E, dtype=torch.int32).pin_memory(), torch.empty(E, dtype=torch.int32).pin_memory()
    h_keep = torch.empty(max(sub.n_hits, 1), dtype=torch.uint8).pin_memory()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    acc = np.zeros(4)
    for r in range(reps + 1):
        ev[0].record(stream)
        dx.copy_(hx, non_blocking=True); dy.copy_(hy, non_blocking=True); do.copy_(ho, non_blocking=True)
        ev[1].record(stream)
        ctx.run_batch(dx, dy, do, peaks, npk, keep, status, stream)
        ev[2].record(stream)
        h_npk.copy_(npk, non_blocking=True); h_st.copy_(status, non_blocking=True)
        h_keep.copy_(keep, non_blocking=True)
        ev[3].record(stream)
        ev[3].synchronize()
        if r:                                   # the first run warms up
            acc += [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3]),
                    ev[0].elapsed_time(ev[3])]
    return [round(float(v), 4) for v in acc / reps]


def _split_kernel_ms(H, wl, sub, cap, reps):
    """Mean time (ms) of hough_run_batch_split over a resident batch, 16-wave workgroups (the
    shape the serving loop gives small batches)."""
    import torch
    ctx = H.Context.for_workload(wl, max_peaks=cap)
    try:
        ctx.set_batch_plan(16, 1, 0)
    except H.HoughError:
        pass
    x, y, off = H.to_device(sub)
    ws = ctx.split_workspace(sub.n_events)
    out = [t for t in ctx.run_batch_split(x, y, off, ws)]
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    total = 0.0
    for _ in range(reps):
        a.record(stream)
        ctx.run_batch_split(x, y, off, ws, *out)
        b.record(stream)
        b.synchronize()
        total += a.elapsed_time(b)
    ctx.close()
    return round(total / reps, 4)


def sweeps(H, wl, ev, reps: int = 10, cpu_budget_s: float = 20.0, plan: dict | None = None):
    """The paper's batch-scale and block-size studies, reshaped for this path (Sec. IV, Fig. 8
    and Fig. 9): (1) runtime against the number of events, GPU end to end (PCIe both ways) and
    kernel only, beside the CPU oracle on the host cores while it fits the budget; (2) per-stage
    times (transfer in, fused kernel, transfer back) against the workgroup size, at the
    1,000-event scale.  Every point is the mean of `reps` runs, as in the paper.  `plan` (a
    batch_plan dict, the benchmark's own launch shape) is used for the events study."""
    from oracle import oracle
    cap = MAX_PEAKS[wl.name]
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1))
    out = {"events": [], "block": [], "reps": reps, "workload": wl.name,
           "cpu": f"oracle, OpenMP over events, {threads} threads"}
    ctx = H.Context.for_workload(wl, max_peaks=cap)
    if plan is not None:
        ctx.set_batch_plan(plan["waves_per_group"], plan["column_groups"], plan["groups_per_cu"])
    out["plan"] = dict(ctx.batch_plan)
    spent, per_event = 0.0, 0.0
    for n in (1, 10, 100, 1000, 10000):
        idx = np.arange(n) % ev.n_events              # past the generated events: repeated ones
        sub = ev.subset(idx)
        h2d, kern, d2h, total = _stage_times(H, ctx, sub, cap, reps)
        row = {"events": n, "gpu_e2e_ms": total, "gpu_kernel_ms": kern, "h2d_ms": h2d, "d2h_ms": d2h}
        if spent + per_event * n * threads < cpu_budget_s:
            t0 = time.perf_counter()
            oracle.run_batch(wl, sub.x, sub.y, sub.offsets, cap=cap, n_threads=threads)
            dt = time.perf_counter() - t0
            spent += dt * threads
            per_event = dt / n
            row["cpu_ms"] = round(dt * 1e3, 3)
            row["speedup_e2e"] = round(dt * 1e3 / total, 1)
        if n <= 100:                                  # small batches: the split (latency) form
            row["gpu_kernel_split_ms"] = _split_kernel_ms(H, wl, sub, cap, reps)
        log(f"sweep events {row}")
        out["events"].append(row)
    sub = ev.subset(np.arange(min(1000, ev.n_events)))
    for waves in (4, 6, 8, 12, 16):
        for groups in (1, 2):
            try:
                ctx.set_batch_plan(waves, groups, 0)
            except H.HoughError:
                continue
            h2d, kern, d2h, total = _stage_times(H, ctx, sub, cap, reps)
            plan = ctx.batch_plan
            row = {"threads_per_workgroup": 64 * waves, "column_groups": groups,
                   "workgroups_per_cu": plan["groups_per_cu"], "h2d_ms": h2d, "kernel_ms": kern,
                   "d2h_ms": d2h, "total_ms": total}
            log(f"sweep block {row}")
            out["block"].append(row)
    ctx.close()
    return out


def serving(H, duration_s: float, warmup_s: float, plain_duration_s: float, pool_events: int = 8192):
    """Open-loop Poisson arrivals of a 50/50 mix of the 1000-event-workload and dense-workload
    generators (pools of `pool_events` each, seed 0) through the native serving loop.  The
    events' hits wait in host memory and each batch's hits go to the device when it is admitted
    (one asynchronous copy per batch), so latency includes that transfer.  Served (continuous
    batching, 8 streams) at each rate; the same with hits already resident in device memory at
    one rate; and the plain per-event launch (its hits sent the same way) under the same kind of
    trace (shorter, it saturates).  Latency = results in host memory - scheduled arrival;
    warm-up arrivals are excluded."""
    from paper_2607_04067_amd import serve
    evs, ctxs = [], []
    for name in ("paper-1000ev-360x256", "dense-2000ev-720x512"):
        wl = synth.WORKLOADS[name]
        log(f"serving pool: {pool_events} events of {name}")
        evs.append(synth.make_events(wl, 0, n_events=pool_events))
        ctxs.append(H.Context.for_workload(wl, max_peaks=MAX_PEAKS[name]))
    host = [serve.Pool(c, e, resident=False) for c, e in zip(ctxs, evs)]
    sizes = [e.n_events for e in evs]
    hits = sum(e.n_hits for e in evs)
    out = {"mix": "50/50 paper-1000ev-360x256 / dense-2000ev-720x512 generators",
           "pool_events": pool_events, "mean_hits": round(hits / sum(sizes), 1),
           "n_streams": 8, "max_batch_events": 256, "small_batch_events": 64, "split_batch_events": 16,
           "hits": "in host memory; each batch's offsets and hits sent in one async copy when admitted",
           "latency": "results (n_peaks, status, keep) in host memory minus scheduled arrival",
           "served": {}, "served_resident": {}, "plain": {}}
    cfg = dict(n_streams=8, max_batch_events=256, max_batch_hits=1 << 21, small_batch_events=64,
               split_batch_events=16)
    for i, rate in enumerate(SERVE_RATES):
        tr = serve.poisson_trace(rate, warmup_s + duration_s, sizes, [0.5, 0.5], seed=100 + i)
        res, _, _ = serve.run(host, tr, **cfg)
        out["served"][str(rate)] = serve.summarize(tr, res, warmup_us=warmup_s * 1e6)
        log(f"served {rate}/s: {out['served'][str(rate)]}")
    resident = [serve.Pool(c, e, resident=True) for c, e in zip(ctxs, evs)]
    rate = SERVE_RATES[2]
    tr = serve.poisson_trace(rate, warmup_s + duration_s / 2, sizes, [0.5, 0.5], seed=102)
    res, _, _ = serve.run(resident, tr, **cfg)
    out["served_resident"][str(rate)] = serve.summarize(tr, res, warmup_us=warmup_s * 1e6)
    log(f"served (resident hits) {rate}/s: {out['served_resident'][str(rate)]}")
    del resident
    for i, rate in enumerate(SERVE_RATES[:2]):
        tr = serve.poisson_trace(rate, plain_duration_s, sizes, [0.5, 0.5], seed=200 + i)
        res, _, _ = serve.run(host, tr, n_streams=8, plain=True, max_batch_hits=1 << 16)
        out["plain"][str(rate)] = serve.summarize(tr, res)
        log(f"plain {rate}/s: {out['plain'][str(rate)]}")
    for c in ctxs:
        c.close()
    return out


PHASE_NAMES = ("pop", "setup", "vote", "peaks", "list", "retain", "finish")


def phase_split(workload: str, plan=None, steps: int = 5) -> dict:
    """Where a fused-kernel workgroup's time goes, from the instrumented build
    (libhough_phases.so, include/hough_debug.h): per-phase shares of the workgroups' summed
    time over `steps` launches, the mean workgroup's busy share of the kernel span, and the LDS
    vote rate while voting (lane-updates per clock per CU, taking a CU's resident workgroups to
    vote at the same time).  Must run in a process that has not loaded libhough.so."""
    import ctypes
    import torch
    from paper_2607_04067_amd import build
    from paper_2607_04067_amd import hough as H
    L = H.load(build.PHASES_LIB)
    L.hough_debug_phase_ticks.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.hough_debug_phase_ticks.restype = ctypes.c_int
    wl = synth.WORKLOADS[workload]
    ev = synth.make_events(wl, 0)
    ctx = H.Context.for_workload(wl, max_peaks=MAX_PEAKS[wl.name])
    if plan:
        ctx.set_batch_plan(*plan)
    xt, yt, ot = H.to_device(ev)
    outs = ctx.run_batch(xt, yt, ot)
    torch.cuda.synchronize()
    ticks = (ctypes.c_uint64 * 9)()
    khz = ctypes.c_uint32(0)
    if L.hough_debug_phase_ticks(ticks, 9, 1, ctypes.byref(khz)) != 0:
        raise RuntimeError("hough_debug_phase_ticks failed")
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        ctx.run_batch(xt, yt, ot, *outs, stream)
    b.record(stream)
    b.synchronize()
    kern_ms = a.elapsed_time(b) / steps
    if L.hough_debug_phase_ticks(ticks, 9, 1, ctypes.byref(khz)) != 0:
        raise RuntimeError("hough_debug_phase_ticks failed")
    t = [int(v) for v in ticks]
    busy = sum(t[:7])
    hz = khz.value * 1e3
    p = ctx.batch_plan
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    grid = min(p["groups_per_cu"] * n_cu, ev.n_events)
    lane_updates = t[8] * 64 * p["column_groups"]
    vote_s = t[2] / hz
    ctx.close()
    return {"workload": workload, "plan": p, "steps": steps, "kernel_ms": round(kern_ms, 4),
            "clock_khz": khz.value, "events": t[7] // steps,
            "share": {n: round(t[i] / busy, 4) for i, n in enumerate(PHASE_NAMES)},
            "workgroup_busy_share": round(busy / hz / (grid * steps * kern_ms / 1e3), 4),
            # lane-updates per second of one voting workgroup, times the workgroups a CU holds
            "vote_lanes_per_clk_per_cu": round(lane_updates / vote_s * p["groups_per_cu"] / CLOCK_HZ, 2),
            "source": kernel_source_id()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(synth.WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's default launch shape instead of autotuning it before timing")
    ap.add_argument("--plan", default=None,
                    help="W,G,C: run this launch shape (waves per workgroup, column groups, workgroups per CU) "
                         "instead of tuning")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch each step eagerly instead of replaying it from a HIP graph")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-e2e", action="store_true", help="skip the PCIe-inclusive measurement")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="measured seconds of arrivals per served rate (after 1 s of warm-up)")
    ap.add_argument("--dedup", action="store_true",
                    help="suppress duplicate hits (HOUGH_FLAG_DEDUP: one more launch per step)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the other configurations' kernel times (the 16-event, 1,000-event, dense "
                         "and paper-grid workloads)")
    ap.add_argument("--no-relative", action="store_true",
                    help="skip the relative-threshold and periodic-grid measurements (their launches share "
                         "the fused kernel's name)")
    ap.add_argument("--sweeps", action="store_true",
                    help="add the runtime-vs-events and stage-times-vs-workgroup-size studies")
    ap.add_argument("--phases", default=None,
                    help="comma-separated workloads: print the fused kernel's phase split from the "
                         "instrumented build (libhough_phases.so) instead of the benchmark")
    ap.add_argument("--copy-reference-mb", type=int, default=0,
                    help="also time a plain device copy of this many MiB (HBM reference for counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path is single-GPU: events are independent, so "
              f"a batch would shard across GPUs with no exchange); got --gpus {args.gpus}", file=sys.stderr)
        return 2

    if args.phases:
        plan = tuple(int(v) for v in args.plan.split(",")) if args.plan else None
        for w in args.phases.split(","):
            log(f"phase split of {w}")
            print(json.dumps({"phases": phase_split(w, plan)}), flush=True)
        return 0

    import torch
    from paper_2607_04067_amd import hough as H

    wl = synth.WORKLOADS[args.workload]
    log(f"generating {wl.n_events} events of {wl.name}")
    ev = synth.make_events(wl, 0)
    votes = ev.n_hits * wl.n_theta
    ctx = H.Context.for_workload(wl, max_peaks=MAX_PEAKS[wl.name], dedup=args.dedup)
    xt, yt, ot = H.to_device(ev)
    E = ev.n_events
    peaks = torch.zeros((E, MAX_PEAKS[wl.name], 2), dtype=torch.int32, device="cuda")
    npk = torch.zeros(E, dtype=torch.int32, device="cuda")
    keep = torch.zeros(ev.n_hits, dtype=torch.uint8, device="cuda")
    status = torch.zeros(E, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    tuned = None
    if args.plan:
        ctx.set_batch_plan(*(int(v) for v in args.plan.split(",")))
    elif not args.no_tune:
        from paper_2607_04067_amd import autotune
        log("autotuning the launch shape")
        tuned = autotune.tune(ctx, xt, yt, ot, (peaks, npk, keep, status),
                              mean_hits=ev.n_hits / max(E, 1), cache=None)
        log(f"tuned plan {ctx.batch_plan}")

    step = lambda: ctx.run_batch(xt, yt, ot, peaks, npk, keep, status, stream)
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        step()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            ctx.run_batch(xt, yt, ot, peaks, npk, keep, status, torch.cuda.current_stream())
        step = graph.replay

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_times = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    kern_ms = float(np.mean(kern_times))
    ms_per_step = wall / args.steps * 1e3
    st = status.cpu().numpy()
    keep_np = keep.cpu().numpy()
    labels = ev.labels
    events_per_s = E / (ms_per_step / 1e3)
    achieved = votes / (kern_ms / 1e3) / 1e9
    cap = MAX_PEAKS[wl.name]
    stored = int(np.minimum(npk.cpu().numpy().astype(np.int64), cap).sum())
    # algorithmic HBM bytes per launch: x, y and offsets in; keep, peak records, n_peaks, status out
    algo_bytes = 8 * ev.n_hits + 4 * (E + 1) + ev.n_hits + 8 * stored + 8 * E
    prof = None if args.dedup else profiled_traffic(wl.name, ctx.batch_plan)   # counters: plain launch only
    ceiling = lds_atomic_ceiling()
    lds_peak = ceiling["lane_updates_per_s"] / 1e9            # Gvote/s: one LDS lane-update per vote at least
    fp32 = achieved * 1e9 * FLOPS_PER_VOTE / 1e12
    plan = ctx.batch_plan
    path = ("hough_run_batch: " + ("duplicate pass, " if args.dedup else "")
            + ("largest-first schedule pass + " if E > plan["groups_per_cu"] * N_CU else "")
            + "persistent fused kernel" + ("" if args.no_graph else ", captured once in a HIP graph and replayed"))
    out = {
        "metric": METRIC, "value": round(events_per_s, 1), "unit": "events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "events": E, "hits": ev.n_hits, "n_theta": wl.n_theta,
                   "n_rho": wl.n_rho, "threshold": wl.threshold, "rho_window": wl.rho_window,
                   "max_peaks": MAX_PEAKS[wl.name], "path": path, "plan": plan,
                   "plan_source": "fixed by --plan" if args.plan else ("library default" if args.no_tune
                                                                       else "autotuned before timing")},
        "gvotes_per_s": round(votes / (ms_per_step / 1e3) / 1e9, 2),
        "kernel_ms": round(kern_ms, 4),
        "kernel_ms_median": round(float(np.median(kern_times)), 4),
        "kernel_ms_span": "HIP events on the launch stream around each step (schedule pass + fused kernel)",
        "roofline": {"bound": "lds_atomic", "achieved": round(achieved, 1), "peak": round(lds_peak, 1),
                     "unit": "Gvote/s", "frac": round(achieved / lds_peak, 4),
                     "traffic": prof["traffic_bytes"] if prof else None,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "k_batch",
                     "peak_source": ceiling["probe"],
                     "lds_lanes_per_clk_per_cu": ceiling["lanes_per_clk_per_cu"],
                     "fp32": {"achieved_tflops": round(fp32, 2), "peak_tflops": FP32_PEAK_TFLOPS,
                              "frac": round(fp32 / FP32_PEAK_TFLOPS, 4),
                              "flops_per_vote": FLOPS_PER_VOTE},
                     "valu_issue": {"peak_gvote_s": round(VOTE_PEAK_PER_S / 1e9, 1), "ops_per_vote": OPS_PER_VOTE,
                                    "frac": round(achieved / (VOTE_PEAK_PER_S / 1e9), 4)},
                     "algorithmic_bytes": algo_bytes,
                     "hbm_algorithmic_gbs": round(algo_bytes / (kern_ms / 1e3) / 1e9, 2),
                     "hbm_frac": round(algo_bytes / (kern_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "lds_atomic": lds_atomic_rate(ev, plan, wl, kern_ms, ceiling["lane_updates_per_s"])},
        "retention": {"R_c": round(float(keep_np.mean()), 4) if keep_np.size else None,
                      "R_s": round(float(keep_np[labels >= 0].mean()), 4) if (labels >= 0).any() else None,
                      "peaks_per_event": round(float(npk.float().mean().item()), 1),
                      "events_flagged": int((st != 0).sum())},
        "paper_context": "paper: 1,000 simulated events in 0.14 s end to end (7,143 events/s) on an "
                         "RTX 5060 Ti with a 1000x1000 grid; different data, grid and GPU",
    }
    if not args.no_secondary:
        out["secondary"] = secondary(H, [w for w in SECONDARY_WORKLOADS if w != wl.name], ceiling,
                                     tune=not args.no_tune)
    if not args.no_relative:
        out["relative_threshold"] = relative_threshold(H, ctx, xt, yt, ot, peaks, npk, keep, status, ev, stream)
        out["periodic_grid"] = periodic_grid(H, wl, ev, xt, yt, ot, stream)
    if tuned is not None:
        out["autotune_ms"] = tuned["ms"]
        out["autotune_pick"] = tuned["plan"]
    if args.sweeps:
        out["sweeps"] = sweeps(H, wl, ev, plan=ctx.batch_plan)
    if args.copy_reference_mb:
        n = args.copy_reference_mb << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(3):
            dst.copy_(src)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b) / 3
        out["copy_reference"] = {"bytes_read": n, "bytes_written": n, "ms": round(ms, 4),
                                 "gbs": round(2 * n / (ms / 1e3) / 1e9, 1)}
        del src, dst
    if not args.no_e2e:
        log("end to end (pinned host buffers, PCIe)")
        out["end_to_end"] = end_to_end(H, ctx, wl, ev)
    if not args.no_serve:
        out["serving"] = serving(H, args.serve_seconds, 1.0, 0.2)
    if not args.no_plain:
        log("plain per-event path")
        out["plain"] = plain_path(H, wl, ev)
        log("plain per-event path with the iterative peak finder")
        out["plain_iterative"] = iterative_path(H, wl, ev)
        log("track finding against the truth")
        out["physics"] = physics(H, wl, ev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, ev)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
