"""Autotuner for the fused batch kernel's launch shape.

The schedule space is the theta-tile width (64 * column_groups columns) times the split of an
event's hits over the waves of a workgroup (waves_per_group) times the number of workgroups
launched per CU (up to what fits; fewer can divide a small batch more evenly over the grid;
more than a whole rho column allows selects a windowed tile, which pays off where the events'
hits reach only part of the rho range).
Every candidate is timed on the caller's resident batch with HIP
events; the three fastest are timed again with more launches, and the fastest of those is kept
unless the context's own shape is within `keep_margin` of it (then the default stays, so that
run-to-run noise does not flip the shape).  Results are cached in a JSON file keyed by device, grid and a
hits-per-event bucket, so that a later context with the same key starts from the tuned shape.
The schedule never changes results, only speed.
"""
from __future__ import annotations

import json
import os

import torch

CANDIDATES = [(w, g, n) for w in (4, 6, 8, 12, 16) for g in (1, 2) for n in (0, 1, 2, 3)]
DEFAULT_CACHE = os.environ.get("HOUGH_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "hough_batch_plans.json"))


def cache_key(ctx, mean_hits: float) -> str:
    dev = torch.cuda.get_device_name(0).replace(" ", "_")
    bucket = 1 << max(0, int(mean_hits).bit_length() - 1)          # power-of-two bucket
    return f"{dev}|{ctx.n_theta}x{ctx.n_rho}|hits~{bucket}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_plan(ctx, args, reps: int = 5, give_up_ms: float | None = None) -> float:
    """Mean milliseconds of one hough_run_batch over `reps` launches (after one warm-up).  A
    warm-up slower than `give_up_ms` is returned as it is (a windowed plan whose window the
    batch's events do not fit sends them all through the slow spill path)."""
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    ctx.run_batch(*args, stream=stream)
    b.record(stream)
    b.synchronize()
    if give_up_ms is not None and a.elapsed_time(b) > give_up_ms:
        return a.elapsed_time(b)
    a.record(stream)
    for _ in range(reps):
        ctx.run_batch(*args, stream=stream)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def tune(ctx, x, y, offsets, outputs, mean_hits: float, cache: str | None = DEFAULT_CACHE,
         reps: int = 5, force: bool = False, keep_margin: float = 0.02) -> dict:
    """Pick the fastest launch shape for this context on the given resident batch.

    outputs = (peaks, n_peaks, keep, status) buffers as accepted by Context.run_batch.
    Returns {"plan": (waves, groups), "ms": {...per candidate...}} and leaves ctx on the winner.
    """
    key = cache_key(ctx, mean_hits)
    table = _load(cache) if cache else {}
    if not force and key in table:
        ctx.set_batch_plan(*table[key]["plan"])
        return table[key]
    args = (x, y, offsets, *outputs)
    d = ctx.batch_plan
    default = f"{d['waves_per_group']}x{d['column_groups']}x{d['groups_per_cu']}"
    results = {}
    for w, g, n in CANDIDATES:
        try:
            ctx.set_batch_plan(w, g, n)
        except RuntimeError:
            continue
        key_c = f"{w}x{g}x{n or ctx.batch_plan['groups_per_cu']}"
        if key_c not in results:
            best = min(results.values(), default=None)
            results[key_c] = round(time_plan(ctx, args, reps, give_up_ms=4.0 * best if best else None), 5)
    finalists = sorted(results, key=results.get)[:3]
    if default in results and default not in finalists:
        finalists.append(default)
    final = {}
    for key_c in finalists:
        ctx.set_batch_plan(*(int(v) for v in key_c.split("x")))
        final[key_c] = round(time_plan(ctx, args, 4 * reps), 5)
    best = min(final, key=final.get)
    if default in final and final[default] <= final[best] * (1.0 + keep_margin):
        best = default
    w, g, n = (int(v) for v in best.split("x"))
    ctx.set_batch_plan(w, g, n)
    entry = {"plan": [w, g, n], "ms": results, "final_ms": final, "default": default}
    if cache:
        table[key] = entry
        os.makedirs(os.path.dirname(cache) or ".", exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return entry
