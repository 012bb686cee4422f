"""The serving loop's scheduler on the host, with no device: hough_serve_simulate runs the same
scheduling core as hough_serve_run (admission, per-kind queues, batch formation, slot choice,
bookkeeping) against a cost model on a simulated clock, so every timing below is exact."""
import numpy as np
import pytest

from paper_2607_04067_amd import serve


def _trace(arrivals, kinds, events=None):
    tr = np.zeros(len(arrivals), serve.REQ_DTYPE)
    tr["arrival_us"] = arrivals
    tr["kind"] = kinds
    tr["event"] = np.arange(len(arrivals)) if events is None else events
    return tr


def _batches(res):
    """(slot, launch_us) -> request indices of each launched batch."""
    out = {}
    for i, r in enumerate(res):
        out.setdefault((int(r["slot"]), float(r["launch_us"])), []).append(i)
    return out


def _cost(m, n, h):
    return m[0] + m[1] * n + m[2] * h


def test_idle_server_launches_on_arrival_and_latency_is_the_modelled_service():
    tr = _trace([0.0, 1000.0, 2000.0], [0, 0, 0])
    hits = np.array([100, 200, 300])
    m = (10.0, 1.0, 0.5)
    res = serve.simulate(tr, hits, [m], n_streams=2)
    assert np.array_equal(res["launch_us"], tr["arrival_us"])
    assert np.allclose(res["done_us"] - res["launch_us"], [_cost(m, 1, h) for h in hits])
    assert np.all(res["batch_events"] == 1)


def test_memory_based_admission_caps_events_and_hits_per_batch():
    rng = np.random.default_rng(1)
    n = 400
    tr = _trace(np.sort(rng.uniform(0, 2000, n)), rng.integers(0, 2, n))
    hits = rng.integers(50, 700, n)
    res = serve.simulate(tr, hits, [(30.0, 0.5, 0.2), (60.0, 1.0, 0.4)], n_streams=3, max_batch_events=16,
                         max_batch_hits=2000)
    for (slot, t), reqs in _batches(res).items():
        assert len(reqs) <= 16
        assert hits[reqs].sum() <= 2000
        assert len(set(tr["kind"][reqs])) == 1            # a batch holds one grid's events
        assert all(res["batch_events"][r] == len(reqs) for r in reqs)
        assert np.all(tr["arrival_us"][reqs] <= t)         # only arrived events are admitted
    assert res["batch_events"].max() > 1                   # events that waited were batched together


def test_full_arena_takes_one_event_per_batch():
    tr = _trace(np.zeros(10), np.zeros(10, np.int64))
    hits = np.full(10, 1000)
    res = serve.simulate(tr, hits, [(5.0, 0.0, 0.01)], n_streams=2, max_batch_events=8, max_batch_hits=1000)
    assert np.all(res["batch_events"] == 1)
    # two slots in turn: requests 0,1 at t=0, 2,3 at 15 us, ...
    assert np.allclose(np.sort(res["launch_us"]), np.repeat(np.arange(5) * 15.0, 2))


def test_fifo_within_a_kind_and_no_starvation_across_kinds():
    """A flood of one kind never holds back the other: a free slot always takes the kind whose
    oldest waiting request arrived first, and each kind's requests launch in arrival order."""
    rng = np.random.default_rng(2)
    n = 3000
    arr = np.sort(rng.uniform(0, 120000, n))     # 25k/s against about 40k/s of capacity
    kinds = (rng.random(n) < 0.03).astype(np.int64)        # kind 1 is rare
    tr = _trace(arr, kinds)
    hits = rng.integers(100, 4000, n)
    m = [(20.0, 0.5, 0.05), (40.0, 1.0, 0.1)]
    res = serve.simulate(tr, hits, m, n_streams=4, max_batch_events=64, max_batch_hits=60000)
    for k in (0, 1):
        sel = np.flatnonzero(kinds == k)
        assert np.all(np.diff(res["launch_us"][sel]) >= 0)
    # bound on any wait: every slot busy with the longest possible batch, twice over; the rare
    # kind waits no longer than the flood does
    longest = max(_cost(mk, 64, 60000) for mk in m)
    wait = res["launch_us"] - tr["arrival_us"]
    assert wait.max() <= 2 * longest
    assert wait[kinds == 1].max() <= wait[kinds == 0].max() + longest
    assert np.all(res["done_us"] > res["launch_us"])


def test_a_slot_never_runs_two_batches_at_once_and_slots_overlap():
    rng = np.random.default_rng(3)
    n = 500
    tr = _trace(np.sort(rng.uniform(0, 5000, n)), np.zeros(n, np.int64))
    hits = rng.integers(500, 3000, n)
    res = serve.simulate(tr, hits, [(50.0, 1.0, 0.1)], n_streams=4, max_batch_events=32, max_batch_hits=40000)
    spans = {}
    for (slot, t), reqs in _batches(res).items():
        spans.setdefault(slot, []).append((t, float(res["done_us"][reqs[0]])))
    assert set(spans) <= {0, 1, 2, 3}
    for s, iv in spans.items():
        iv.sort()
        assert all(a[1] <= b[0] for a, b in zip(iv, iv[1:])), s     # back to back at most
    # at some moment more than one slot is busy (continuous batching overlaps batches)
    allv = sorted(iv for v in spans.values() for iv in v)
    assert any(b[0] < a[1] for a, b in zip(allv, allv[1:]))


def test_partial_batch_is_held_for_max_wait_then_launched():
    tr = _trace([0.0, 10.0, 20.0, 500.0], [0, 0, 0, 0])
    hits = np.array([100, 100, 100, 100])
    res = serve.simulate(tr, hits, [(5.0, 0.0, 0.0)], n_streams=1, max_batch_events=8, max_wait_us=100.0)
    assert np.allclose(res["launch_us"][:3], 100.0) and np.all(res["batch_events"][:3] == 3)
    assert res["launch_us"][3] == pytest.approx(600.0) and res["batch_events"][3] == 1
    # a batch that fills before the deadline goes at once
    res = serve.simulate(tr, hits, [(5.0, 0.0, 0.0)], n_streams=1, max_batch_events=3, max_wait_us=100.0)
    assert np.allclose(res["launch_us"][:3], 20.0)


def test_plain_mode_runs_one_event_per_slot():
    tr = _trace(np.zeros(6), np.zeros(6, np.int64))
    res = serve.simulate(tr, np.full(6, 10), [(7.0, 0.0, 0.0)], n_streams=2, plain=True)
    assert np.all(res["batch_events"] == 1)
    assert np.allclose(np.sort(res["done_us"]), np.repeat([7.0, 14.0, 21.0], 2))


def test_latency_accounting_under_saturation_matches_a_closed_form():
    """One slot, requests every 10 us, each batch 25 us + 1 us per event: the queue grows, each
    batch takes everything that waited, and every request's completion equals the launch of its
    batch plus that batch's modelled cost."""
    n = 200
    tr = _trace(np.arange(n) * 10.0, np.zeros(n, np.int64))
    hits = np.full(n, 100)
    m = (25.0, 1.0, 0.0)
    res = serve.simulate(tr, hits, [m], n_streams=1, max_batch_events=1000, max_batch_hits=1 << 30)
    t, i = 0.0, 0
    while i < n:
        waiting = [j for j in range(i, n) if tr["arrival_us"][j] <= t] or [i]
        t = max(t, tr["arrival_us"][waiting[0]])
        waiting = [j for j in range(i, n) if tr["arrival_us"][j] <= t]
        done = t + _cost(m, len(waiting), 0)
        assert np.allclose(res["launch_us"][waiting], t) and np.allclose(res["done_us"][waiting], done)
        i += len(waiting)
        t = done


def test_invalid_traces_are_refused():
    from paper_2607_04067_amd import hough
    m = [(1.0, 0.0, 0.0)]
    with pytest.raises(hough.HoughError):           # an event larger than a slot's arena
        serve.simulate(_trace([0.0], [0]), np.array([5000]), m, max_batch_hits=4000)
    with pytest.raises(hough.HoughError):           # arrivals out of order
        serve.simulate(_trace([5.0, 1.0], [0, 0]), np.array([1, 1]), m)
    with pytest.raises(hough.HoughError):           # a kind without a model
        serve.simulate(_trace([0.0], [1]), np.array([1]), m)
    with pytest.raises(hough.HoughError):           # more than 32 streams
        serve.simulate(_trace([0.0], [0]), np.array([1]), m, n_streams=33)
    with pytest.raises(hough.HoughError):           # a batch that costs nothing
        serve.simulate(_trace([0.0], [0]), np.array([1]), [(0.0, 0.0, 0.0)])


def test_summary_splits_the_tail_into_waiting_and_service():
    """A simulated stall: one slot, steady arrivals, and a burst that queues behind one long
    batch; the summary's tail is that episode, its latency mostly waiting."""
    n = 2000
    arr = np.arange(n) * 50.0
    arr[1000:1040] = arr[1000]                       # a burst of 40 requests at once
    tr = _trace(np.sort(arr), np.zeros(n, np.int64))
    hits = np.full(n, 100)
    res = serve.simulate(tr, hits, [(20.0, 30.0, 0.0)], n_streams=1, max_batch_events=4, max_batch_hits=1 << 20)
    s = serve.summarize(tr, res)
    assert s["requests"] == n and s["max_us"] >= s["p99_9_us"] >= s["p99_us"] >= s["p50_us"]
    assert s["max_wait_us"] >= s["p99_9_wait_us"] and s["max_service_us"] >= s["p99_9_service_us"]
    tail = s["tail"]
    assert tail["requests"] >= 2
    assert tail["mean_wait_us"] > tail["mean_service_us"]           # queued behind the burst
    lo, hi = tail["arrival_ms"]
    assert 49.0 <= lo <= hi <= 53.0                                   # the burst at 50 ms
    assert 49.0 <= tail["worst_arrival_ms"] <= 53.0
