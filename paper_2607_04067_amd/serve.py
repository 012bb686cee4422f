"""Serving: an open-loop arrival trace run through the native request loop (hough_serve_run).

Events of each kind sit in a device-resident CSR pool (one per grid).  A trace draws arrival
times from a Poisson process and, per arrival, a kind (Bernoulli mix) and a pool event; the C++
loop admits, batches, launches and completes them (see include/hough_serve.h).  This module only
builds the inputs, calls the library and summarises the per-request timings.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import hough


class hough_serve_pool(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("host_offsets", ctypes.c_void_p), ("n_events", ctypes.c_uint32)]


class hough_serve_config(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_batch_events", ctypes.c_int32),
                ("max_batch_hits", ctypes.c_int32), ("plain", ctypes.c_int32), ("copy_peaks", ctypes.c_int32),
                ("small_batch_events", ctypes.c_int32), ("split_batch_events", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("max_wait_us", ctypes.c_double)]


REQ_DTYPE = np.dtype([("arrival_us", "<f8"), ("kind", "<i4"), ("event", "<u4")])
RES_DTYPE = np.dtype([("launch_us", "<f8"), ("done_us", "<f8"), ("n_peaks", "<u4"), ("status", "<u4"),
                      ("batch_events", "<u4"), ("pad", "<u4")])


def _lib():
    L = hough.load()
    if not hasattr(L, "_serve_ready"):
        L.hough_serve_run.argtypes = [ctypes.POINTER(hough_serve_pool), ctypes.c_int32,
                                      ctypes.POINTER(hough_serve_config), ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
        L.hough_serve_run.restype = ctypes.c_int
        L._serve_ready = True
    return L


class Pool:
    """A resident event pool: device hits + offsets, a host copy of the offsets, and its context."""

    def __init__(self, ctx: hough.Context, batch):
        self.ctx = ctx
        self.batch = batch
        self.x, self.y, self.offsets = hough.to_device(batch)
        self.host_offsets = np.ascontiguousarray(batch.offsets, dtype=np.uint32)

    def struct(self) -> hough_serve_pool:
        return hough_serve_pool(self.ctx._ctx.value, self.x.data_ptr(), self.y.data_ptr(),
                                self.offsets.data_ptr(), self.host_offsets.ctypes.data, self.batch.n_events)


def poisson_trace(rate_hz: float, duration_s: float, pool_sizes, mix, seed: int = 0) -> np.ndarray:
    """Arrivals of a Poisson process of `rate_hz` over `duration_s`; each picks a kind with
    probabilities `mix` and a uniformly random event of that kind's pool."""
    rng = np.random.default_rng(seed)
    n = int(rate_hz * duration_s * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n)) * 1e6
    t = t[t < duration_s * 1e6]
    kinds = rng.choice(len(mix), size=t.size, p=np.asarray(mix) / np.sum(mix))
    sizes = np.asarray(pool_sizes, dtype=np.float64)
    events = np.minimum((rng.random(t.size) * sizes[kinds]).astype(np.int64), sizes[kinds].astype(np.int64) - 1)
    tr = np.zeros(t.size, REQ_DTYPE)
    tr["arrival_us"], tr["kind"], tr["event"] = t, kinds, events
    return tr


def run(pools, trace: np.ndarray, n_streams: int = 8, max_batch_events: int = 256,
        max_batch_hits: int = 1 << 20, plain: bool = False, copy_peaks: bool = False,
        max_wait_us: float = 0.0, want_keep: bool = False, want_peaks: int = 0,
        small_batch_events: int = 64, split_batch_events: int = 16):
    """Run `trace` to completion; returns (results array, keep bytes or None, peaks or None)."""
    L = _lib()
    structs = (hough_serve_pool * len(pools))(*[p.struct() for p in pools])
    cfg = hough_serve_config(int(n_streams), int(max_batch_events), int(max_batch_hits), int(plain),
                             int(copy_peaks or want_peaks > 0), int(small_batch_events), int(split_batch_events), 0, float(max_wait_us))
    trace = np.ascontiguousarray(trace, dtype=REQ_DTYPE)
    res = np.zeros(trace.size, RES_DTYPE)
    keep = peaks = None
    if want_keep:
        hits = sum(int(pools[k].host_offsets[e + 1] - pools[k].host_offsets[e]) for k, e in
                   zip(trace["kind"], trace["event"]))
        keep = np.zeros(max(hits, 1), np.uint8)
    if want_peaks:
        peaks = np.zeros((max(trace.size, 1), want_peaks, 2), np.uint32)
    torch.cuda.synchronize()
    rc = L.hough_serve_run(structs, len(pools), ctypes.byref(cfg), trace.ctypes.data, trace.size,
                           res.ctypes.data, keep.ctypes.data if keep is not None else None,
                           peaks.ctypes.data if peaks is not None else None, int(want_peaks))
    if rc != hough.HOUGH_OK:
        raise hough.HoughError(rc, "hough_serve_run")
    return res, keep, peaks


def summarize(trace: np.ndarray, res: np.ndarray, warmup_us: float = 0.0) -> dict:
    """p50/p99 latency (done - scheduled arrival), its split into waiting for a launch and the
    launch-to-results service time, and the sustained rate over the measured window."""
    sel = trace["arrival_us"] >= warmup_us
    if not sel.any():
        return {}
    lat = res["done_us"][sel] - trace["arrival_us"][sel]
    wait = res["launch_us"][sel] - trace["arrival_us"][sel]
    span = (res["done_us"][sel].max() - trace["arrival_us"][sel].min()) / 1e6
    return {"requests": int(sel.sum()), "p50_us": round(float(np.percentile(lat, 50)), 1),
            "p99_us": round(float(np.percentile(lat, 99)), 1), "max_us": round(float(lat.max()), 1),
            "p50_wait_us": round(float(np.percentile(wait, 50)), 1),
            "p50_service_us": round(float(np.percentile(lat - wait, 50)), 1),
            "events_per_s": round(float(sel.sum() / span), 1) if span > 0 else None,
            "mean_batch": round(float(res["batch_events"][sel].mean()), 2)}
