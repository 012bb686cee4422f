"""hough_run_batch_split_static (the library's static scratch in place of a caller workspace)
gives hough_run_batch_split's results bit for bit, on two calls in a row, the second smaller,
and refuses a batch whose workspace exceeds the scratch before enqueueing anything."""
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


def _outputs(ctx, E, n_keep, fill=0):
    import torch
    mp = ctx.params.max_peaks
    return dict(peaks=torch.full((E, mp, 2), -1, dtype=torch.int32, device="cuda"),
                n_peaks=torch.full((E,), -1, dtype=torch.int32, device="cuda"),
                keep=torch.full((n_keep,), fill, dtype=torch.uint8, device="cuda"),
                status=torch.full((E,), -1, dtype=torch.int32, device="cuda"))


def _same(ref, out, E, mp):
    import torch
    pk_r, n_r, keep_r, st_r = ref
    pk_o, n_o, keep_o, st_o = out
    assert torch.equal(n_r[:E], n_o[:E]) and torch.equal(st_r[:E], st_o[:E]) and torch.equal(keep_r, keep_o)
    n = torch.clamp(n_r[:E], max=mp).cpu().numpy()
    a, b = pk_r.cpu().numpy(), pk_o.cpu().numpy()
    for e in range(E):
        assert np.array_equal(a[e, :n[e]], b[e, :n[e]]), e


@pytest.mark.parametrize("name,sizes", [("dense-2000ev-720x512", (12, 5)), ("paper-1000ev-360x256", (40, 3)),
                                        ("paper-1000ev-1000x1000", (6, 1))])
def test_static_split_equals_split(H, name, sizes):
    import torch
    wl = synth.WORKLOADS[name]
    ctx = H.Context.for_workload(wl, max_peaks=4096)
    ctx.set_batch_plan(16, 1, 0)
    for call, E in enumerate(sizes):
        ev = synth.make_events(wl, 11 + call, n_events=E)
        xt, yt, ot = H.to_device(ev)
        say(f"static split {name}: call {call}, {E} events, {ev.n_hits} hits")
        ws = ctx.split_workspace(E)
        ref = ctx.run_batch_split(xt, yt, ot, ws, **_outputs(ctx, E, ev.n_hits))
        out = ctx.run_batch_split_static(xt, yt, ot, **_outputs(ctx, E, ev.n_hits, fill=0xAB))
        torch.cuda.synchronize()
        _same(ref, out, E, ctx.params.max_peaks)
        assert int(ws.count_nonzero()) == 0
    ctx.close()


def test_static_split_gather_form_two_calls(H):
    """The gather form (pool ids, keep offsets with a gap) on the static scratch, a larger then a
    smaller batch, each equal to the caller-workspace form's results."""
    import torch
    wl = synth.WORKLOADS["paper-1000ev-360x256"]
    pool = synth.make_events(wl, 0, n_events=40)
    ctx = H.Context.for_workload(wl, max_peaks=8192)
    xt, yt, ot = H.to_device(pool)
    for ids in (np.array([7, 3, 3, 39, 0, 21, 7, 12, 30, 31], np.int64), np.array([5, 38], np.int64)):
        sub = pool.subset(ids)
        koff = (sub.offsets[:-1] + 5).astype(np.int32)
        n_keep = sub.n_hits + 9
        E = len(ids)
        say(f"static split gather ids={ids.tolist()}")
        ws = ctx.split_workspace(E)
        ref = ctx.run_batch_split(xt, yt, ot, ws, event_ids=_t(ids.astype(np.int32)), keep_offsets=_t(koff),
                                  keep_size=n_keep, **{k: v for k, v in _outputs(ctx, E, n_keep, 0xAB).items()})
        out = ctx.run_batch_split_static(xt, yt, ot, event_ids=_t(ids.astype(np.int32)), keep_offsets=_t(koff),
                                         keep_size=n_keep, **_outputs(ctx, E, n_keep, 0xAB))
        torch.cuda.synchronize()
        _same(ref, out, E, ctx.params.max_peaks)
    ctx.close()


def test_static_split_refuses_batches_beyond_the_scratch(H):
    import torch
    wl = synth.WORKLOADS["paper-1000ev-1000x1000"]
    ctx = H.Context.for_workload(wl, max_peaks=64)
    lib = H.load()
    E = 1
    while lib.hough_split_workspace_bytes(ctx._ctx, E) <= H.STATIC_SCRATCH_BYTES:
        E *= 2
    ev = synth.make_events(wl, 3, n_events=2)
    xt, yt, ot = H.to_device(ev)
    offs = torch.zeros(E + 1, dtype=torch.int32, device="cuda")     # E empty events
    with pytest.raises(H.HoughError) as ei:
        ctx.run_batch_split_static(xt, yt, offs, **_outputs(ctx, E, ev.n_hits))
    assert ei.value.status == H.HOUGH_ETOOLARGE
    # the context still works afterwards
    out = ctx.run_batch_split_static(xt, yt, ot, **_outputs(ctx, 2, ev.n_hits))
    ref = ctx.run_batch_split(xt, yt, ot, ctx.split_workspace(2), **_outputs(ctx, 2, ev.n_hits))
    torch.cuda.synchronize()
    _same(ref, out, 2, ctx.params.max_peaks)
    ctx.close()
