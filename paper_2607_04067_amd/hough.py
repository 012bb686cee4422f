"""ctypes binding of libhough.so (see include/hough.h for the exact semantics).

This module only marshals arguments: it checks that tensors live on the GPU with the right
dtype and layout, passes their device pointers and torch's current HIP stream to the C ABI,
and decodes results.  Every step of the method runs in the library's HIP kernels; there is no
fallback, and loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhough.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "hough.h")

HOUGH_OK, HOUGH_EINVAL, HOUGH_ENOMEM, HOUGH_EOVERFLOW, HOUGH_EDEVICE, HOUGH_ETOOLARGE = 0, -1, -2, -3, -4, -5
STATIC_SCRATCH_BYTES = 32 << 20     # HOUGH_STATIC_SCRATCH_BYTES
ACC_U16, ACC_I32 = 1, 2
EV_PEAKS_TRUNCATED, EV_INVALID_HITS, EV_TOO_MANY_HITS = 1, 2, 4
EV_DEDUP_SKIPPED = 16


class HoughError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what} failed: {status_string(status)} ({status})")
        self.status = status


class hough_batch_plan(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_int32), ("column_groups", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("lds_bytes", ctypes.c_int32), ("window_rows", ctypes.c_int32)]


class hough_params(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int32), ("n_rho", ctypes.c_int32),
                ("rho_min", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("acc_type", ctypes.c_int32), ("threshold", ctypes.c_int32),
                ("rho_window", ctypes.c_int32), ("max_peaks", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


FLAG_THETA_PERIODIC = 1
FLAG_DEDUP = 2


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhough.so (raises if it is not built; nothing runs without it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2607_04067_amd.build`")
    L = ctypes.CDLL(path)
    vp, u32, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
    L.hough_config.argtypes = [ctypes.POINTER(hough_params), ctypes.POINTER(vp)]
    L.hough_config.restype = i32
    L.hough_destroy.argtypes = [vp]
    L.hough_destroy.restype = None
    L.hough_get_params.argtypes = [vp, ctypes.POINTER(hough_params)]
    L.hough_get_params.restype = i32
    L.hough_vote.argtypes = [vp, vp, vp, u32, vp, vp]
    L.hough_vote.restype = i32
    L.hough_peaks.argtypes = [vp, vp, vp, u32, vp, vp]
    L.hough_peaks.restype = i32
    L.hough_peaks_iterative.argtypes = [vp, vp, u32, u32, ctypes.c_int32, ctypes.c_int32, vp, u32, vp, vp, vp]
    L.hough_peaks_iterative.restype = i32
    L.hough_track_params.argtypes = [vp, vp, vp, u32, vp, vp, u32, ctypes.c_double, vp, vp]
    L.hough_track_params.restype = i32
    L.hough_max_dedup_hits.argtypes = []
    L.hough_max_dedup_hits.restype = u32
    L.hough_run_batch_relative.argtypes = [vp, vp, vp, vp, u32, u32, u32, vp, vp, vp, vp, vp]
    L.hough_run_batch_relative.restype = i32
    L.hough_iterative_workspace_bytes.argtypes = [vp, u32]
    L.hough_iterative_workspace_bytes.restype = ctypes.c_size_t
    L.hough_run_batch_iterative.argtypes = [vp, vp, vp, vp, u32, u32, u32, ctypes.c_int32, ctypes.c_int32,
                                            vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.hough_run_batch_iterative.restype = i32
    L.hough_retain.argtypes = [vp, vp, vp, u32, vp, vp, u32, vp, vp]
    L.hough_retain.restype = i32
    L.hough_run_batch.argtypes = [vp, vp, vp, vp, u32, vp, vp, vp, vp, vp]
    L.hough_run_batch.restype = i32
    L.hough_run_batch_gather.argtypes = [vp, vp, vp, vp, vp, vp, u32, vp, vp, vp, vp, vp]
    L.hough_run_batch_gather.restype = i32
    L.hough_run_batch_split.argtypes = [vp, vp, vp, vp, vp, vp, u32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.hough_run_batch_split.restype = i32
    L.hough_run_batch_split_static.argtypes = [vp, vp, vp, vp, vp, vp, u32, vp, vp, vp, vp, vp]
    L.hough_run_batch_split_static.restype = i32
    L.hough_split_workspace_bytes.argtypes = [vp, u32]
    L.hough_split_workspace_bytes.restype = ctypes.c_size_t
    L.hough_get_batch_plan.argtypes = [vp, ctypes.POINTER(hough_batch_plan)]
    L.hough_get_batch_plan.restype = i32
    L.hough_set_batch_plan.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.hough_set_batch_plan.restype = i32
    L.hough_max_batch_hits.argtypes = [vp]
    L.hough_max_batch_hits.restype = u32
    L.hough_max_n_rho.argtypes = []
    L.hough_max_n_rho.restype = ctypes.c_int32
    L.hough_status_string.argtypes = [i32]
    L.hough_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def status_string(status: int) -> str:
    return load().hough_status_string(int(status)).decode()


def header_functions(path: str = HEADER_PATH) -> list[str]:
    """Names of the functions include/hough.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hough_[a-z_0-9]+)\s*\(", text)))


def _check(rc: int, what: str):
    if rc != HOUGH_OK:
        raise HoughError(rc, what)


def _dev(t: torch.Tensor, dtype, name: str, numel: int | None = None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")
    return t.data_ptr()


def _hits(x: torch.Tensor, y: torch.Tensor, keep: torch.Tensor | None = None, keep_needed: int | None = None) -> int:
    """Number of hits of x and y, after checking that y holds as many as x and that keep (when
    given) has room for keep_needed bytes (one per hit by default).  Raises ValueError before any
    pointer reaches the library: a short buffer would be read or written out of bounds there."""
    n = x.numel()
    if y.numel() != n:
        raise ValueError(f"x and y differ in length ({n} and {y.numel()})")
    if keep is not None:
        need = n if keep_needed is None else int(keep_needed)
        if keep.numel() < need:
            raise ValueError(f"keep needs at least {need} bytes, has {keep.numel()}")
    return n


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def decode_peaks(peaks: torch.Tensor | np.ndarray, n: int | None = None) -> np.ndarray:
    """hough_peak records (int32 pairs) -> int64 array [n, 3] of (theta_bin, rho_bin, count)."""
    a = peaks.detach().cpu().numpy() if isinstance(peaks, torch.Tensor) else np.asarray(peaks)
    a = a.reshape(-1, 2).view(np.uint32)
    if n is not None:
        a = a[:n]
    return np.stack([a[:, 0] & 0xFFFF, a[:, 0] >> 16, a[:, 1]], axis=1).astype(np.int64)


# hough_track records: 5 doubles, int32 charge, uint32 n_hits (48 bytes)
TRACK_DTYPE = np.dtype([("a", "<f8"), ("b", "<f8"), ("radius", "<f8"), ("pt", "<f8"), ("phi_c", "<f8"),
                        ("charge", "<i4"), ("n_hits", "<u4")])


def decode_tracks(tracks: torch.Tensor | np.ndarray, n: int | None = None) -> np.ndarray:
    """hough_track records (a float64 tensor of 6 per record) -> numpy structured array."""
    a = tracks.detach().cpu().numpy() if isinstance(tracks, torch.Tensor) else np.asarray(tracks)
    a = np.ascontiguousarray(a).reshape(-1).view(np.uint8).view(TRACK_DTYPE)
    return a[:n] if n is not None else a


class Context:
    """One configured (theta, rho) grid on the current GPU (wraps hough_ctx)."""

    def __init__(self, n_theta: int, n_rho: int, rho_min: float, rho_max: float, acc_type: str = "i32",
                 threshold: int = 1, rho_window: int = 1, max_peaks: int = 0, periodic: bool = False,
                 dedup: bool = False):
        self._lib = load()
        self.params = hough_params(int(n_theta), int(n_rho), float(rho_min), float(rho_max),
                                   ACC_U16 if acc_type == "u16" else ACC_I32, int(threshold),
                                   int(rho_window), int(max_peaks),
                                   (FLAG_THETA_PERIODIC if periodic else 0) | (FLAG_DEDUP if dedup else 0), 0)
        self.acc_type = acc_type
        self._ctx = ctypes.c_void_p()
        _check(self._lib.hough_config(ctypes.byref(self.params), ctypes.byref(self._ctx)), "hough_config")
        self._dummy = torch.zeros(8, dtype=torch.int32, device="cuda")

    @classmethod
    def for_workload(cls, wl, max_peaks: int = 4096, threshold: int | None = None,
                     rho_window: int | None = None, periodic: bool = False, dedup: bool = False) -> "Context":
        return cls(wl.n_theta, wl.n_rho, wl.rho_min, wl.rho_max, wl.acc,
                   wl.threshold if threshold is None else threshold,
                   wl.rho_window if rho_window is None else rho_window, max_peaks, periodic, dedup)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self._lib.hough_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_theta(self) -> int:
        return self.params.n_theta

    @property
    def n_rho(self) -> int:
        return self.params.n_rho

    @property
    def max_batch_hits(self) -> int:
        return int(self._lib.hough_max_batch_hits(self._ctx))

    @property
    def batch_plan(self) -> dict:
        p = hough_batch_plan()
        _check(self._lib.hough_get_batch_plan(self._ctx, ctypes.byref(p)), "hough_get_batch_plan")
        return {"waves_per_group": p.waves_per_group, "column_groups": p.column_groups,
                "groups_per_cu": p.groups_per_cu, "lds_bytes": p.lds_bytes, "window_rows": p.window_rows}

    def set_batch_plan(self, waves_per_group: int, column_groups: int, groups_per_cu: int = 0) -> None:
        _check(self._lib.hough_set_batch_plan(self._ctx, int(waves_per_group), int(column_groups),
                                              int(groups_per_cu)), "hough_set_batch_plan")

    def _ptr_or_dummy(self, t: torch.Tensor, dtype, name: str) -> int:
        if t.numel() == 0:
            return self._dummy.data_ptr()
        return _dev(t, dtype, name)

    # ------------------------------------------------------------------ plain path
    def vote(self, x: torch.Tensor, y: torch.Tensor, acc: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Accumulator [n_theta, n_rho] (int32, or int16 holding uint16 bits) of one event."""
        n = _hits(x, y)
        dt = torch.int16 if self.acc_type == "u16" else torch.int32
        if acc is None:
            acc = torch.empty((self.n_theta, self.n_rho), dtype=dt, device=x.device)
        pa = _dev(acc, dt, "acc", self.n_theta * self.n_rho)
        px = self._ptr_or_dummy(x, torch.float32, "x")
        py = self._ptr_or_dummy(y, torch.float32, "y")
        _check(self._lib.hough_vote(self._ctx, px, py, n, pa, _stream(stream)), "hough_vote")
        return acc

    def peaks(self, acc: torch.Tensor, cap: int, peaks: torch.Tensor | None = None,
              n_peaks: torch.Tensor | None = None, stream=None):
        """(peaks int32 [cap, 2] hough_peak records, n_peaks int32 [1] true count)."""
        dt = torch.int16 if self.acc_type == "u16" else torch.int32
        pa = _dev(acc, dt, "acc", self.n_theta * self.n_rho)
        if peaks is None:
            peaks = torch.zeros((max(cap, 1), 2), dtype=torch.int32, device=acc.device)
        if n_peaks is None:
            n_peaks = torch.zeros(1, dtype=torch.int32, device=acc.device)
        pp = _dev(peaks, torch.int32, "peaks", 2 * cap)
        pn = _dev(n_peaks, torch.int32, "n_peaks", 1)
        _check(self._lib.hough_peaks(self._ctx, pa, pp, int(cap), pn, _stream(stream)), "hough_peaks")
        return peaks, n_peaks

    def peaks_iterative(self, acc: torch.Tensor, cap: int, frac=(1, 2), r_theta: int = 5, r_rho: int = 5,
                        peaks: torch.Tensor | None = None, n_peaks: torch.Tensor | None = None,
                        status: torch.Tensor | None = None, stream=None):
        """The paper's peak finder: (peaks int32 [cap, 2] in extraction order, n_peaks int32 [1],
        status int32 [1])."""
        dt = torch.int16 if self.acc_type == "u16" else torch.int32
        pa = _dev(acc, dt, "acc", self.n_theta * self.n_rho)
        if peaks is None:
            peaks = torch.zeros((max(cap, 1), 2), dtype=torch.int32, device=acc.device)
        if n_peaks is None:
            n_peaks = torch.zeros(1, dtype=torch.int32, device=acc.device)
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=acc.device)
        pp = _dev(peaks, torch.int32, "peaks", 2 * cap)
        pn = _dev(n_peaks, torch.int32, "n_peaks", 1)
        ps = _dev(status, torch.int32, "status", 1)
        _check(self._lib.hough_peaks_iterative(self._ctx, pa, int(frac[0]), int(frac[1]), int(r_theta),
                                               int(r_rho), pp, int(cap), pn, ps, _stream(stream)),
               "hough_peaks_iterative")
        return peaks, n_peaks, status

    def track_params(self, x: torch.Tensor, y: torch.Tensor, peaks: torch.Tensor, n_peaks: torch.Tensor,
                     cap: int, b_tesla: float = 1.0, tracks: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
        """Candidate circles of the first min(n_peaks, cap) peaks: float64 [cap, 6] holding
        hough_track records (decode with decode_tracks)."""
        _hits(x, y)
        if tracks is None:
            tracks = torch.zeros((max(cap, 1), 6), dtype=torch.float64, device=peaks.device)
        pt = _dev(tracks, torch.float64, "tracks", 6 * cap)
        pp = _dev(peaks, torch.int32, "peaks", 2 * cap)
        pn = _dev(n_peaks, torch.int32, "n_peaks", 1)
        px = self._ptr_or_dummy(x, torch.float32, "x")
        py = self._ptr_or_dummy(y, torch.float32, "y")
        _check(self._lib.hough_track_params(self._ctx, px, py, x.numel(), pp, pn, int(cap), float(b_tesla),
                                            pt, _stream(stream)), "hough_track_params")
        return tracks

    def retain(self, x: torch.Tensor, y: torch.Tensor, peaks: torch.Tensor, n_peaks: torch.Tensor, cap: int,
               keep: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        n = _hits(x, y, keep)
        if keep is None:
            keep = torch.empty(n, dtype=torch.uint8, device=x.device)
        pk = self._ptr_or_dummy(keep, torch.uint8, "keep")
        pp = _dev(peaks, torch.int32, "peaks", 2 * cap)
        pn = _dev(n_peaks, torch.int32, "n_peaks", 1)
        px = self._ptr_or_dummy(x, torch.float32, "x")
        py = self._ptr_or_dummy(y, torch.float32, "y")
        _check(self._lib.hough_retain(self._ctx, px, py, n, pp, pn, int(cap), pk, _stream(stream)),
               "hough_retain")
        return keep

    # ----------------------------------------------------------------- fused batch
    def run_batch(self, x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, peaks: torch.Tensor | None = None,
                  n_peaks: torch.Tensor | None = None, keep: torch.Tensor | None = None,
                  status: torch.Tensor | None = None, stream=None, frac=None):
        """Whole path over CSR events.  offsets: int32 [E+1] (uint32 values).  frac=(num, den):
        each event's threshold relative to its largest count (hough_run_batch_relative).
        Returns (peaks int32 [E, max_peaks, 2], n_peaks int32 [E], keep uint8 [H], status int32 [E])."""
        _hits(x, y, keep)
        E = offsets.numel() - 1
        mp = self.params.max_peaks
        dev = offsets.device
        if peaks is None:
            peaks = torch.zeros((max(E, 1), max(mp, 1), 2), dtype=torch.int32, device=dev)
        if n_peaks is None:
            n_peaks = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        if status is None:
            status = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        if keep is None:
            keep = torch.zeros(x.numel(), dtype=torch.uint8, device=dev)
        po = _dev(offsets, torch.int32, "offsets", E + 1)
        pp = _dev(peaks, torch.int32, "peaks", 2 * E * mp) if mp > 0 else 0
        pn = _dev(n_peaks, torch.int32, "n_peaks", E)
        ps = _dev(status, torch.int32, "status", E)
        pk = self._ptr_or_dummy(keep, torch.uint8, "keep")
        px = self._ptr_or_dummy(x, torch.float32, "x")
        py = self._ptr_or_dummy(y, torch.float32, "y")
        if frac is None:
            _check(self._lib.hough_run_batch(self._ctx, px, py, po, E, pp, pn, pk, ps, _stream(stream)),
                   "hough_run_batch")
        else:
            _check(self._lib.hough_run_batch_relative(self._ctx, px, py, po, E, int(frac[0]), int(frac[1]),
                                                      pp, pn, pk, ps, _stream(stream)), "hough_run_batch_relative")
        return peaks, n_peaks, keep, status


    def iterative_workspace(self, n_events: int) -> torch.Tensor:
        """Device workspace for run_batch_iterative over up to n_events events."""
        n = int(self._lib.hough_iterative_workspace_bytes(self._ctx, int(n_events)))
        return torch.empty(max(n, 256), dtype=torch.uint8, device="cuda")

    def run_batch_iterative(self, x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, frac=(1, 2),
                            r_theta: int = 5, r_rho: int = 5, workspace: torch.Tensor | None = None,
                            peaks: torch.Tensor | None = None, n_peaks: torch.Tensor | None = None,
                            keep: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None):
        """The paper's peak finder over CSR events (hough_run_batch_iterative).  Returns (peaks
        int32 [E, max_peaks, 2] in extraction order, n_peaks int32 [E], keep uint8 [H],
        status int32 [E])."""
        _hits(x, y, keep)
        E = offsets.numel() - 1
        mp = self.params.max_peaks
        dev = offsets.device
        if workspace is None:
            workspace = self.iterative_workspace(E)
        if peaks is None:
            peaks = torch.zeros((max(E, 1), max(mp, 1), 2), dtype=torch.int32, device=dev)
        if n_peaks is None:
            n_peaks = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        if status is None:
            status = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        if keep is None:
            keep = torch.zeros(x.numel(), dtype=torch.uint8, device=dev)
        po = _dev(offsets, torch.int32, "offsets", E + 1)
        pp = _dev(peaks, torch.int32, "peaks", 2 * E * mp) if mp > 0 else 0
        pn = _dev(n_peaks, torch.int32, "n_peaks", E)
        ps = _dev(status, torch.int32, "status", E)
        pw = _dev(workspace, torch.uint8, "workspace")
        pk = self._ptr_or_dummy(keep, torch.uint8, "keep")
        px = self._ptr_or_dummy(x, torch.float32, "x")
        py = self._ptr_or_dummy(y, torch.float32, "y")
        _check(self._lib.hough_run_batch_iterative(self._ctx, px, py, po, E, int(frac[0]), int(frac[1]),
                                                   int(r_theta), int(r_rho), pp, pn, pk, ps, pw,
                                                   workspace.numel(), _stream(stream)),
               "hough_run_batch_iterative")
        return peaks, n_peaks, keep, status

    def split_workspace(self, n_events: int) -> torch.Tensor:
        """A zero-filled device workspace for run_batch_split over up to n_events events."""
        n = int(self._lib.hough_split_workspace_bytes(self._ctx, int(n_events)))
        return torch.zeros(max(n, 256), dtype=torch.uint8, device="cuda")

    def run_batch_split(self, x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor,
                        workspace: torch.Tensor | None = None, peaks: torch.Tensor | None = None,
                        n_peaks: torch.Tensor | None = None, keep: torch.Tensor | None = None,
                        status: torch.Tensor | None = None, event_ids: torch.Tensor | None = None,
                        keep_offsets: torch.Tensor | None = None, keep_size: int | None = None, stream=None):
        """run_batch's (or, with event_ids and keep_offsets, run_batch_gather's) results, computed
        with each event's theta tiles on separate workgroups (the latency form).
        workspace: from split_workspace (kept zero between calls)."""
        return self._split(x, y, offsets, workspace, peaks, n_peaks, keep, status, event_ids, keep_offsets,
                           keep_size, stream, static=False)

    def run_batch_split_static(self, x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor,
                               peaks: torch.Tensor | None = None, n_peaks: torch.Tensor | None = None,
                               keep: torch.Tensor | None = None, status: torch.Tensor | None = None,
                               event_ids: torch.Tensor | None = None, keep_offsets: torch.Tensor | None = None,
                               keep_size: int | None = None, stream=None):
        """run_batch_split on the library's static scratch (hough_run_batch_split_static): the
        call allocates nothing when every output tensor is given."""
        return self._split(x, y, offsets, None, peaks, n_peaks, keep, status, event_ids, keep_offsets,
                           keep_size, stream, static=True)

    def _split(self, x, y, offsets, workspace, peaks, n_peaks, keep, status, event_ids, keep_offsets,
               keep_size, stream, static: bool):
        if (event_ids is None) != (keep_offsets is None):
            raise ValueError("event_ids and keep_offsets go together")
        if event_ids is not None and keep_size is None:
            raise ValueError("the gather form needs keep_size (the keep bytes the batch writes)")
        _hits(x, y, keep, x.numel() if event_ids is None else keep_size)
        E = offsets.numel() - 1 if event_ids is None else event_ids.numel()
        mp = self.params.max_peaks
        dev = offsets.device
        if workspace is None and not static:
            workspace = self.split_workspace(E)
        if peaks is None:
            peaks = torch.zeros((max(E, 1), max(mp, 1), 2), dtype=torch.int32, device=dev)
        if n_peaks is None:
            n_peaks = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        if status is None:
            status = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        if keep is None:
            n_keep = x.numel() if event_ids is None else int(keep_size or 0)
            keep = torch.zeros(max(n_keep, 1), dtype=torch.uint8, device=dev)
        if event_ids is None:
            po = _dev(offsets, torch.int32, "offsets", E + 1)
            pi = pko = None
        else:
            po = _dev(offsets, torch.int32, "offsets")
            pi = _dev(event_ids, torch.int32, "event_ids", E) if E else self._dummy.data_ptr()
            pko = _dev(keep_offsets, torch.int32, "keep_offsets", E) if E else self._dummy.data_ptr()
        pp = _dev(peaks, torch.int32, "peaks", 2 * E * mp) if mp > 0 else 0
        pn = _dev(n_peaks, torch.int32, "n_peaks", E)
        ps = _dev(status, torch.int32, "status", E)
        pk = self._ptr_or_dummy(keep, torch.uint8, "keep")
        px = self._ptr_or_dummy(x, torch.float32, "x")
        py = self._ptr_or_dummy(y, torch.float32, "y")
        if static:
            _check(self._lib.hough_run_batch_split_static(self._ctx, px, py, po, pi, pko, E, pp, pn, pk, ps,
                                                          _stream(stream)), "hough_run_batch_split_static")
        else:
            pw = _dev(workspace, torch.uint8, "workspace")
            _check(self._lib.hough_run_batch_split(self._ctx, px, py, po, pi, pko, E, pp, pn, pk, ps, pw,
                                                   workspace.numel(), _stream(stream)), "hough_run_batch_split")
        return peaks, n_peaks, keep, status

    def run_batch_gather(self, x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, event_ids: torch.Tensor,
                         keep_offsets: torch.Tensor, peaks: torch.Tensor | None = None,
                         n_peaks: torch.Tensor | None = None, keep: torch.Tensor | None = None,
                         status: torch.Tensor | None = None, keep_size: int | None = None, stream=None):
        """hough_run_batch over pool events `event_ids` (int32, uint32 values); event e's keep
        bytes start at keep_offsets[e] (int32).  keep_size: bytes of keep the batch writes (checked
        against keep when both are given).  Returns (peaks, n_peaks, keep, status)."""
        if keep_size is None:
            raise ValueError("the gather form needs keep_size (the keep bytes the batch writes)")
        _hits(x, y, keep, keep_size)
        E = event_ids.numel()
        mp = self.params.max_peaks
        dev = offsets.device
        if peaks is None:
            peaks = torch.zeros((max(E, 1), max(mp, 1), 2), dtype=torch.int32, device=dev)
        if n_peaks is None:
            n_peaks = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        if status is None:
            status = torch.zeros(max(E, 1), dtype=torch.int32, device=dev)
        if keep is None:
            keep = torch.zeros(max(int(keep_size or 0), 1), dtype=torch.uint8, device=dev)
        po = _dev(offsets, torch.int32, "offsets")
        pi = _dev(event_ids, torch.int32, "event_ids", E) if E else self._dummy.data_ptr()
        pko = _dev(keep_offsets, torch.int32, "keep_offsets", E) if E else self._dummy.data_ptr()
        pp = _dev(peaks, torch.int32, "peaks", 2 * E * mp) if mp > 0 else 0
        pn = _dev(n_peaks, torch.int32, "n_peaks", E)
        ps = _dev(status, torch.int32, "status", E)
        pk = self._ptr_or_dummy(keep, torch.uint8, "keep")
        px = self._ptr_or_dummy(x, torch.float32, "x")
        py = self._ptr_or_dummy(y, torch.float32, "y")
        _check(self._lib.hough_run_batch_gather(self._ctx, px, py, po, pi, pko, E, pp, pn, pk, ps,
                                                _stream(stream)), "hough_run_batch_gather")
        return peaks, n_peaks, keep, status


def to_device(batch, device="cuda"):
    """Move an EventBatch's hits and offsets to the GPU (x, y float32; offsets int32)."""
    x = torch.from_numpy(np.ascontiguousarray(batch.x)).to(device)
    y = torch.from_numpy(np.ascontiguousarray(batch.y)).to(device)
    off = torch.from_numpy(batch.offsets.astype(np.int64).astype(np.int32)).to(device)
    return x, y, off
