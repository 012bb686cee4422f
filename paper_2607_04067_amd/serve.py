"""Serving: an open-loop arrival trace run through the native request loop (hough_serve_run).

Events of each kind sit in a CSR pool (one per grid), either resident in device memory or in
host memory (then each batch's hits are sent to the device when it is admitted).  A trace draws
arrival times from a Poisson process and, per arrival, a kind (Bernoulli mix) and a pool event;
the C++ loop admits, batches, launches and completes them (see include/hough_serve.h).
simulate() replays the same scheduling against a cost model on a simulated clock
(hough_serve_simulate), without a device.  This module only builds the inputs, calls the
library and summarises the per-request timings.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import hough


class hough_serve_pool(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("host_offsets", ctypes.c_void_p), ("n_events", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("host_x", ctypes.c_void_p), ("host_y", ctypes.c_void_p)]


class hough_serve_model(ctypes.Structure):
    _fields_ = [("fixed_us", ctypes.c_double), ("per_event_us", ctypes.c_double), ("per_hit_us", ctypes.c_double)]


class hough_serve_config(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_batch_events", ctypes.c_int32),
                ("max_batch_hits", ctypes.c_int32), ("plain", ctypes.c_int32), ("copy_peaks", ctypes.c_int32),
                ("small_batch_events", ctypes.c_int32), ("split_batch_events", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("max_wait_us", ctypes.c_double)]


REQ_DTYPE = np.dtype([("arrival_us", "<f8"), ("kind", "<i4"), ("event", "<u4")])
RES_DTYPE = np.dtype([("launch_us", "<f8"), ("done_us", "<f8"), ("n_peaks", "<u4"), ("status", "<u4"),
                      ("batch_events", "<u4"), ("slot", "<u4")])


def _lib():
    L = hough.load()
    if not hasattr(L, "_serve_ready"):
        L.hough_serve_run.argtypes = [ctypes.POINTER(hough_serve_pool), ctypes.c_int32,
                                      ctypes.POINTER(hough_serve_config), ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
        L.hough_serve_run.restype = ctypes.c_int
        L.hough_serve_simulate.argtypes = [ctypes.c_int32, ctypes.POINTER(hough_serve_config), ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(hough_serve_model),
                                           ctypes.c_void_p]
        L.hough_serve_simulate.restype = ctypes.c_int
        L._serve_ready = True
    return L


class Pool:
    """An event pool and its context.  resident=True: hits and offsets in device memory (the
    loop sends only event indices); resident=False: hits in host memory, sent with each batch
    (the host arrays are kept here so that they outlive the run)."""

    def __init__(self, ctx: hough.Context, batch, resident: bool = True):
        self.ctx = ctx
        self.batch = batch
        self.resident = resident
        self.host_offsets = np.ascontiguousarray(batch.offsets, dtype=np.uint32)
        if resident:
            self.x, self.y, self.offsets = hough.to_device(batch)
        else:
            self.host_x = np.ascontiguousarray(batch.x, dtype=np.float32)
            self.host_y = np.ascontiguousarray(batch.y, dtype=np.float32)

    def struct(self) -> hough_serve_pool:
        if self.resident:
            return hough_serve_pool(self.ctx._ctx.value, self.x.data_ptr(), self.y.data_ptr(),
                                    self.offsets.data_ptr(), self.host_offsets.ctypes.data, self.batch.n_events,
                                    0, None, None)
        return hough_serve_pool(self.ctx._ctx.value, None, None, None, self.host_offsets.ctypes.data,
                                self.batch.n_events, 0, self.host_x.ctypes.data, self.host_y.ctypes.data)


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


def simulate(trace: np.ndarray, hits: np.ndarray, models, n_streams: int = 8, max_batch_events: int = 256,
             max_batch_hits: int = 1 << 20, plain: bool = False, max_wait_us: float = 0.0,
             small_batch_events: int = 0, split_batch_events: int = 0) -> np.ndarray:
    """The serving loop's scheduling of `trace` on a simulated clock (hough_serve_simulate):
    hits[i] is request i's event size, models[kind] = (fixed_us, per_event_us, per_hit_us) the
    cost of a batch of that kind.  Returns the per-request results array (no device used)."""
    L = _lib()
    cfg = hough_serve_config(int(n_streams), int(max_batch_events), int(max_batch_hits), int(plain), 0,
                             int(small_batch_events), int(split_batch_events), 0, float(max_wait_us))
    trace = np.ascontiguousarray(trace, dtype=REQ_DTYPE)
    hits = np.ascontiguousarray(hits, dtype=np.uint32)
    if hits.size != trace.size:
        raise ValueError("one hit count per request")
    ms = (hough_serve_model * max(len(models), 1))(*[hough_serve_model(*map(float, m)) for m in models])
    res = np.zeros(trace.size, RES_DTYPE)
    rc = L.hough_serve_simulate(len(models), ctypes.byref(cfg), trace.ctypes.data, hits.ctypes.data, trace.size,
                                ms, res.ctypes.data)
    if rc != hough.HOUGH_OK:
        raise hough.HoughError(rc, "hough_serve_simulate")
    return res


def summarize(trace: np.ndarray, res: np.ndarray, warmup_us: float = 0.0) -> dict:
    """p50/p99/p99.9 latency (done - scheduled arrival), its split into waiting for a launch and
    the launch-to-results service time, and the sustained rate over the measured window.  "tail"
    describes the requests at or above the p99.9 latency: how much of their latency was waiting
    and how much service, their batch sizes, and the arrival-time span they come from (one short
    span: a single episode, such as a stall of the host loop; spread over the run: load)."""
    sel = trace["arrival_us"] >= warmup_us
    if not sel.any():
        return {}
    arr = trace["arrival_us"][sel]
    lat = res["done_us"][sel] - arr
    wait = res["launch_us"][sel] - arr
    serv = lat - wait
    span = (res["done_us"][sel].max() - arr.min()) / 1e6
    r1 = lambda v: round(float(v), 1)
    p999 = np.percentile(lat, 99.9)
    t = lat >= p999
    tail = {"requests": int(t.sum()), "mean_wait_us": r1(wait[t].mean()), "mean_service_us": r1(serv[t].mean()),
            "mean_batch": round(float(res["batch_events"][sel][t].mean()), 2),
            "arrival_ms": [r1(arr[t].min() / 1e3), r1(arr[t].max() / 1e3)],
            "worst_arrival_ms": r1(arr[np.argmax(lat)] / 1e3)}
    return {"requests": int(sel.sum()), "p50_us": r1(np.percentile(lat, 50)),
            "p99_us": r1(np.percentile(lat, 99)), "p99_9_us": r1(p999), "max_us": r1(lat.max()),
            "p50_wait_us": r1(np.percentile(wait, 50)), "p99_9_wait_us": r1(np.percentile(wait, 99.9)),
            "max_wait_us": r1(wait.max()),
            "p50_service_us": r1(np.percentile(serv, 50)), "p99_9_service_us": r1(np.percentile(serv, 99.9)),
            "max_service_us": r1(serv.max()),
            "events_per_s": r1(sel.sum() / span) if span > 0 else None,
            "mean_batch": round(float(res["batch_events"][sel].mean()), 2), "tail": tail}
