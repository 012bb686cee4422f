"""Host-only checks of the binding's argument validation and of hough_config's error paths.

No GPU is needed: the binding validates tensor lengths before any pointer reaches the library,
and hough_config rejects bad parameters (and reports an allocation failure through its test
hook) before its first HIP call.
"""
import ctypes
import os

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_04067_amd", "libhough.so")


@pytest.fixture(scope="module")
def H():
    if not os.path.exists(LIB):
        from paper_2607_04067_amd import build
        build.build()
    from paper_2607_04067_amd import hough
    return hough


def _offline_context(H, n_theta=8, n_rho=8, max_peaks=4):
    """A Context whose validation runs but which holds no library handle: any call that got past
    the argument checks would fail on the missing handle instead of reaching a kernel."""
    ctx = H.Context.__new__(H.Context)
    ctx.params = H.hough_params(n_theta, n_rho, -0.005, 0.005, H.ACC_I32, 1, 1, max_peaks, 0, 0)
    ctx.acc_type = "i32"
    ctx._ctx = ctypes.c_void_p()
    ctx._lib = None
    return ctx


def _f(n):
    return torch.zeros(n, dtype=torch.float32)


def test_short_y_is_rejected_by_every_entry_point(H):
    ctx = _offline_context(H)
    x, y = _f(10), _f(9)
    off = torch.tensor([0, 10], dtype=torch.int32)
    pk = torch.zeros((4, 2), dtype=torch.int32)
    npk = torch.zeros(1, dtype=torch.int32)
    calls = [lambda: ctx.vote(x, y),
             lambda: ctx.retain(x, y, pk, npk, 4),
             lambda: ctx.track_params(x, y, pk, npk, 4),
             lambda: ctx.run_batch(x, y, off),
             lambda: ctx.run_batch_iterative(x, y, off),
             lambda: ctx.run_batch_split(x, y, off),
             lambda: ctx.run_batch_gather(x, y, off, torch.zeros(1, dtype=torch.int32),
                                          torch.zeros(1, dtype=torch.int32), keep_size=10)]
    for call in calls:
        with pytest.raises(ValueError, match="differ in length"):
            call()


def test_short_keep_is_rejected(H):
    ctx = _offline_context(H)
    x, y = _f(10), _f(10)
    off = torch.tensor([0, 10], dtype=torch.int32)
    pk = torch.zeros((4, 2), dtype=torch.int32)
    npk = torch.zeros(1, dtype=torch.int32)
    short = torch.zeros(9, dtype=torch.uint8)
    calls = [lambda: ctx.retain(x, y, pk, npk, 4, keep=short),
             lambda: ctx.run_batch(x, y, off, keep=short),
             lambda: ctx.run_batch_iterative(x, y, off, keep=short),
             lambda: ctx.run_batch_split(x, y, off, keep=short),
             # gather form: the caller states how many keep bytes the batch writes
             lambda: ctx.run_batch_gather(x, y, off, torch.zeros(1, dtype=torch.int32),
                                          torch.zeros(1, dtype=torch.int32), keep=short, keep_size=12),
             lambda: ctx.run_batch_split(x, y, off, keep=short, event_ids=torch.zeros(1, dtype=torch.int32),
                                         keep_offsets=torch.zeros(1, dtype=torch.int32), keep_size=12)]
    for call in calls:
        with pytest.raises(ValueError, match="keep needs at least"):
            call()
    # the gather forms cannot check keep without being told how many bytes the batch writes
    ids = torch.zeros(1, dtype=torch.int32)
    for call in [lambda: ctx.run_batch_gather(x, y, off, ids, ids, keep=short),
                 lambda: ctx.run_batch_split(x, y, off, keep=short, event_ids=ids, keep_offsets=ids)]:
        with pytest.raises(ValueError, match="keep_size"):
            call()


def test_host_tensors_are_rejected_after_the_length_checks(H):
    """Lengths that agree pass the first check; the host tensors are then refused as not on the
    device, still before the library is called."""
    ctx = _offline_context(H)
    x, y = _f(10), _f(10)
    off = torch.tensor([0, 10], dtype=torch.int32)
    with pytest.raises(ValueError, match="CUDA"):
        ctx.run_batch(x, y, off, keep=torch.zeros(10, dtype=torch.uint8))


def _params(H, **kw):
    p = dict(n_theta=360, n_rho=256, rho_min=-1 / 200, rho_max=1 / 200, acc_type=H.ACC_I32, threshold=10,
             rho_window=1, max_peaks=16, flags=0, reserved=0)
    p.update(kw)
    return H.hough_params(*p.values())


def test_config_reports_allocation_failure(H, monkeypatch):
    """HOUGH_TEST_FAIL_ALLOC=1 makes hough_config fail as an allocation would: HOUGH_ENOMEM and
    no context."""
    L = H.load()
    monkeypatch.setenv("HOUGH_TEST_FAIL_ALLOC", "1")
    out = ctypes.c_void_p(12345)
    assert L.hough_config(ctypes.byref(_params(H)), ctypes.byref(out)) == H.HOUGH_ENOMEM
    assert out.value is None


@pytest.mark.parametrize("bad", [dict(n_theta=0), dict(n_rho=0), dict(n_theta=70000), dict(rho_min=0.01),
                                 dict(rho_max=float("nan")), dict(acc_type=3), dict(threshold=0),
                                 dict(rho_window=-1), dict(max_peaks=-1), dict(flags=64), dict(reserved=1),
                                 dict(flags=1, rho_min=-0.004)])
def test_config_rejects_bad_parameters_before_any_device_call(H, bad):
    L = H.load()
    out = ctypes.c_void_p()
    assert L.hough_config(ctypes.byref(_params(H, **bad)), ctypes.byref(out)) == H.HOUGH_EINVAL
    assert out.value is None
    assert L.hough_config(None, ctypes.byref(out)) == H.HOUGH_EINVAL
