"""Python access to the CPU oracle (oracle/hough_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the benchmark's CPU
baseline leg.  The product path never imports this module.  It shares no code with the HIP
library: the C file builds its own tables and applies the binning rule itself.

The functions mirror the steps of the method (see the C file's header for the rules):
  Grid        uniform (theta, rho) discretisation constants (Sec. II)
  conformal() Eq. (1)
  rho_bin()   the bin index of rho = u cos(theta_j) + v sin(theta_j) for one hit and column (Sec. II)
  bins()      the same for every hit and column: the binned parameter matrix R of Sec. III
  vote()      accumulator (Sec. II, Sec. III)
  peaks()     threshold + 3x3 local maxima in raster order (Sec. II)
  retain()    per-hit keep mask (Sec. I, Sec. II)
  run_batch() all of the above over CSR-packed events
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hough_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
             "-fopenmp", "-Wall", "-Wextra"]


def build(out: str = _LIB, extra_flags=()) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", *GCC_FLAGS, *extra_flags, "-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def lib():
    """The loaded oracle.  HOUGH_ORACLE_LIB names another build of the same source to load
    instead (the sanitizer build of the tests)."""
    global _lib
    if _lib is None:
        path = os.environ.get("HOUGH_ORACLE_LIB") or _LIB
        if path == _LIB and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(path)
        c_int, c_long, c_double, c_float = ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_float
        L.oracle_tables.argtypes = [c_int, c_int, c_double, c_double, _f32p, _f32p, ctypes.POINTER(c_float)]
        L.oracle_tables.restype = c_int
        L.oracle_conformal.argtypes = [c_float, c_float, ctypes.POINTER(c_float), ctypes.POINTER(c_float)]
        L.oracle_conformal.restype = c_int
        L.oracle_rho_bin.argtypes = [c_float, c_float, c_float, c_float, c_float, c_int]
        L.oracle_rho_bin.restype = c_int
        L.oracle_bins.argtypes = [c_int, c_int, _f32p, _f32p, c_float, _f32p, _f32p, c_long, _i32p]
        L.oracle_bins.restype = None
        L.oracle_vote.argtypes = [c_int, c_int, _f32p, _f32p, c_float, _f32p, _f32p, c_long, _i32p]
        L.oracle_vote.restype = None
        L.oracle_is_peak.argtypes = [_i32p, c_int, c_int, c_int, c_int, c_int]
        L.oracle_is_peak.restype = c_int
        L.oracle_peaks.argtypes = [_i32p, c_int, c_int, c_int, _i32p, _i32p, _i32p, c_long]
        L.oracle_peaks.restype = c_long
        L.oracle_peaks_mode.argtypes = [_i32p, c_int, c_int, c_int, c_int, _i32p, _i32p, _i32p, c_long]
        L.oracle_peaks_mode.restype = c_long
        L.oracle_is_peak_periodic.argtypes = [_i32p, c_int, c_int, c_int, c_int, c_int]
        L.oracle_is_peak_periodic.restype = c_int
        L.oracle_peaks_iterative.argtypes = [_i32p, c_int, c_int, c_int, c_int, c_int, c_int, c_int,
                                             _i32p, _i32p, _i32p, c_long]
        L.oracle_peaks_iterative.restype = c_long
        L.oracle_peaks_iterative_sorted.argtypes = L.oracle_peaks_iterative.argtypes
        L.oracle_peaks_iterative_sorted.restype = c_long
        L.oracle_run_batch_iterative.argtypes = [c_int, c_int, c_double, c_double, c_int, c_int, c_int, c_int,
                                                 c_int, c_int, _f32p, _f32p, _u32p, c_long, c_long, _i32p, _i64p,
                                                 _u8p, c_int, c_int]
        L.oracle_run_batch_iterative.restype = c_int
        _f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        L.oracle_track_params.argtypes = [c_int, c_int, c_double, c_double, _f32p, _f32p, c_float, c_int,
                                          c_double, _f32p, _f32p, c_long, _i32p, _i32p, c_long, _f64p]
        L.oracle_track_params.restype = None
        L.oracle_retain.argtypes = [c_int, _f32p, _f32p, c_float, c_int, _f32p, _f32p, c_long,
                                    _i32p, _i32p, c_long, _u8p]
        L.oracle_retain.restype = None
        L.oracle_run_batch.argtypes = [c_int, c_int, c_double, c_double, c_int, c_int, _f32p, _f32p,
                                       _u32p, c_long, c_long, _i32p, _i64p, _u8p, c_int, c_int, c_int, c_int,
                                       c_int]
        L.oracle_first_copies.argtypes = [_f32p, _f32p, c_long, _u8p]
        L.oracle_vote_dedup.argtypes = [c_int, c_int, _f32p, _f32p, c_float, _f32p, _f32p, c_long, _i32p]
        L.oracle_run_batch.restype = c_int
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = c_int
        _lib = L
    return _lib


class Grid:
    """The (theta, rho) grid and its binning constants, as the oracle computes them."""

    def __init__(self, n_theta: int, n_rho: int, rho_min: float, rho_max: float):
        self.n_theta, self.n_rho = int(n_theta), int(n_rho)
        self.rho_min, self.rho_max = float(rho_min), float(rho_max)
        self.C = np.zeros(self.n_theta, np.float32)
        self.S = np.zeros(self.n_theta, np.float32)
        b = ctypes.c_float()
        if lib().oracle_tables(self.n_theta, self.n_rho, self.rho_min, self.rho_max, self.C, self.S,
                               ctypes.byref(b)) != 0:
            raise ValueError("invalid grid")
        self.B = np.float32(b.value)

    @classmethod
    def of(cls, wl) -> "Grid":
        return cls(wl.n_theta, wl.n_rho, wl.rho_min, wl.rho_max)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def conformal(x: float, y: float):
    """Eq. (1) for one hit: (valid, u, v)."""
    u, v = ctypes.c_float(), ctypes.c_float()
    ok = lib().oracle_conformal(float(np.float32(x)), float(np.float32(y)), ctypes.byref(u), ctypes.byref(v))
    return bool(ok), np.float32(u.value), np.float32(v.value)


def rho_bin(g: Grid, u, v, j: int) -> int:
    return int(lib().oracle_rho_bin(float(u), float(v), float(g.C[j]), float(g.S[j]), float(g.B), g.n_rho))


def bins(g: Grid, x, y) -> np.ndarray:
    """Bin index of rho_ij for every hit i and column j ([H, n_theta]; -1 = no vote)."""
    x, y = _f32(x), _f32(y)
    out = np.zeros((x.size, g.n_theta), np.int32)
    if x.size:
        lib().oracle_bins(g.n_theta, g.n_rho, g.C, g.S, float(g.B), x, y, x.size, out)
    return out


def vote(g: Grid, x, y) -> np.ndarray:
    x, y = _f32(x), _f32(y)
    acc = np.zeros((g.n_theta, g.n_rho), np.int32)
    lib().oracle_vote(g.n_theta, g.n_rho, g.C, g.S, float(g.B), x, y, x.size, acc)
    return acc


def first_copies(x, y) -> np.ndarray:
    """uint8 per hit: 1 iff no earlier hit has bit-identical (x, y) (duplicate suppression)."""
    x, y = _f32(x), _f32(y)
    first = np.zeros(max(x.size, 1), np.uint8)
    lib().oracle_first_copies(x if x.size else np.zeros(1, np.float32),
                              y if y.size else np.zeros(1, np.float32), x.size, first)
    return first[:x.size]


def vote_dedup(g: Grid, x, y) -> np.ndarray:
    """Accumulator with only the first copy of bit-identical hits voting."""
    x, y = _f32(x), _f32(y)
    acc = np.zeros((g.n_theta, g.n_rho), np.int32)
    lib().oracle_vote_dedup(g.n_theta, g.n_rho, g.C, g.S, float(g.B),
                            x if x.size else np.zeros(1, np.float32),
                            y if y.size else np.zeros(1, np.float32), x.size, acc)
    return acc


def peaks(acc: np.ndarray, threshold: int, cap: int | None = None, periodic: bool = False):
    """All peaks (or the first `cap`) in raster order: (j, k, count) arrays and the true count.
    periodic: theta-periodic grid (column n_theta - 1 borders column 0 with rho reversed)."""
    acc = np.ascontiguousarray(acc, dtype=np.int32)
    nt, nr = acc.shape
    cap = nt * nr if cap is None else int(cap)
    pj = np.zeros(max(cap, 1), np.int32); pk = np.zeros_like(pj); pc = np.zeros_like(pj)
    n = int(lib().oracle_peaks_mode(acc, nt, nr, int(threshold), int(bool(periodic)), pj, pk, pc, cap))
    m = min(n, cap)
    return pj[:m].copy(), pk[:m].copy(), pc[:m].copy(), n


def peaks_iterative(acc: np.ndarray, t_abs: int, frac: tuple[int, int], r_theta: int, r_rho: int,
                    cap: int | None = None, sorted_form: bool = False):
    """The paper's peak finder (Sec. II): threshold max(t_abs, ceil(max * frac)), then the
    largest remaining cell (raster-first among equals) is taken and its (2 r_theta + 1) x
    (2 r_rho + 1) neighbourhood suppressed, repeatedly.  (j, k, count) in extraction order and
    the true count.  sorted_form: the same extraction computed by one walk over the sorted
    candidates (oracle_peaks_iterative_sorted), for accumulators with many candidates and peaks."""
    acc = np.ascontiguousarray(acc, dtype=np.int32)
    nt, nr = acc.shape
    cap = nt * nr if cap is None else int(cap)
    pj = np.zeros(max(cap, 1), np.int32); pk = np.zeros_like(pj); pc = np.zeros_like(pj)
    f = lib().oracle_peaks_iterative_sorted if sorted_form else lib().oracle_peaks_iterative
    n = int(f(acc, nt, nr, int(t_abs), int(frac[0]), int(frac[1]), int(r_theta), int(r_rho), pj, pk, pc, cap))
    if n < 0:
        raise MemoryError("oracle_peaks_iterative")
    m = min(n, cap)
    return pj[:m].copy(), pk[:m].copy(), pc[:m].copy(), n


TRACK_FIELDS = ("a", "b", "radius", "pt", "phi_c", "charge", "n_hits")


def track_params(g: Grid, x, y, pj, pk, rho_window: int = 1, b_tesla: float = 1.0) -> np.ndarray:
    """Candidate circle and track parameters of each peak (Eq. (2) with the factor two of
    Eq. (1)): float64 [n_peaks, 7] with columns TRACK_FIELDS (mm, mm, mm, GeV/c, rad, +-1/0,
    hits associated with the peak)."""
    x, y = _f32(x), _f32(y)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    pk = np.ascontiguousarray(pk, dtype=np.int32)
    out = np.zeros((max(pj.size, 1), 7), np.float64)
    lib().oracle_track_params(g.n_theta, g.n_rho, g.rho_min, g.rho_max, g.C, g.S, float(g.B),
                              int(rho_window), float(b_tesla), x, y, x.size, pj, pk, pj.size, out)
    return out[:pj.size].copy()


def is_peak(acc: np.ndarray, threshold: int, j: int, k: int, periodic: bool = False) -> bool:
    acc = np.ascontiguousarray(acc, dtype=np.int32)
    f = lib().oracle_is_peak_periodic if periodic else lib().oracle_is_peak
    return bool(f(acc, acc.shape[0], acc.shape[1], int(threshold), int(j), int(k)))


def retain(g: Grid, x, y, pj, pk, rho_window: int = 1) -> np.ndarray:
    x, y = _f32(x), _f32(y)
    pj = np.ascontiguousarray(pj, np.int32); pk = np.ascontiguousarray(pk, np.int32)
    keep = np.zeros(x.size, np.uint8)
    lib().oracle_retain(g.n_rho, g.C, g.S, float(g.B), int(rho_window), x, y, x.size, pj, pk, pj.size, keep)
    return keep


def run_batch(wl_or_grid, x, y, offsets, threshold: int | None = None, rho_window: int | None = None,
              cap: int = 4096, n_threads: int = 1, periodic: bool = False, dedup: bool = False,
              frac: tuple[int, int] | None = None):
    """Whole path over CSR events.  Returns (peaks[E, cap, 3] as (j, k, count), n_peaks[E], keep[H]).
    dedup: only the first copy of bit-identical hits of an event votes.  frac=(num, den): each
    event's threshold is max(threshold, ceil(its largest count * num / den))."""
    if isinstance(wl_or_grid, Grid):
        g = wl_or_grid
        if threshold is None or rho_window is None:
            raise ValueError("threshold and rho_window are required with a Grid")
    else:
        wl = wl_or_grid
        g = Grid.of(wl)
        threshold = wl.threshold if threshold is None else threshold
        rho_window = wl.rho_window if rho_window is None else rho_window
    x, y = _f32(x), _f32(y)
    offsets = np.ascontiguousarray(offsets, np.uint32)
    E = offsets.size - 1
    out = np.zeros((max(E, 1), max(cap, 1), 3), np.int32)
    n_peaks = np.zeros(max(E, 1), np.int64)
    keep = np.zeros(max(x.size, 1), np.uint8)
    rc = lib().oracle_run_batch(g.n_theta, g.n_rho, g.rho_min, g.rho_max, int(threshold), int(rho_window),
                                x if x.size else np.zeros(1, np.float32), y if y.size else np.zeros(1, np.float32),
                                offsets, E, int(cap), out, n_peaks, keep, int(n_threads), int(bool(periodic)),
                                int(bool(dedup)), int(frac[0]) if frac else 0, int(frac[1]) if frac else 0)
    if rc != 0:
        raise MemoryError("oracle_run_batch failed")
    return out[:E], n_peaks[:E], keep[:x.size]


def run_batch_iterative(g: Grid, x, y, offsets, t_abs: int, frac: tuple[int, int], r_theta: int, r_rho: int,
                        rho_window: int, cap: int, dedup: bool = False):
    """The paper's finder over CSR events, one event at a time: vote (only first copies with
    dedup), iterative extraction (Sec. II, reading of the relative threshold and suppression),
    then retention with the event's first min(n, cap) peaks.  Returns (peaks[E, cap, 3] as
    (j, k, count) in extraction order, n[E], keep[H])."""
    x, y = _f32(x), _f32(y)
    offsets = np.asarray(offsets, np.int64)
    E = offsets.size - 1
    out = np.zeros((max(E, 1), max(cap, 1), 3), np.int32)
    n = np.zeros(max(E, 1), np.int64)
    keep = np.zeros(max(x.size, 1), np.uint8)
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        acc = vote_dedup(g, x[a:b], y[a:b]) if dedup else vote(g, x[a:b], y[a:b])
        pj, pk, pc, m = peaks_iterative(acc, t_abs, frac, r_theta, r_rho, cap=max(cap, 1))
        k = min(m, cap)
        n[e] = m
        out[e, :k] = np.stack([pj[:k], pk[:k], pc[:k]], 1)
        keep[a:b] = retain(g, x[a:b], y[a:b], pj[:k], pk[:k], rho_window)
    return out[:E], n[:E], keep[:x.size]


def run_batch_iterative_fast(g: Grid, x, y, offsets, t_abs: int, frac: tuple[int, int], r_theta: int,
                             r_rho: int, rho_window: int, cap: int, dedup: bool = False, n_threads: int = 1):
    """run_batch_iterative computed in C over n_threads OpenMP threads, with the finder in its
    order form; the same results (a CPU test compares the two)."""
    x, y = _f32(x), _f32(y)
    offsets = np.ascontiguousarray(offsets, np.uint32)
    E = offsets.size - 1
    out = np.zeros((max(E, 1), max(cap, 1), 3), np.int32)
    n = np.zeros(max(E, 1), np.int64)
    keep = np.zeros(max(x.size, 1), np.uint8)
    rc = lib().oracle_run_batch_iterative(g.n_theta, g.n_rho, g.rho_min, g.rho_max, int(t_abs), int(frac[0]),
                                          int(frac[1]), int(r_theta), int(r_rho), int(rho_window),
                                          x if x.size else np.zeros(1, np.float32),
                                          y if y.size else np.zeros(1, np.float32), offsets, E, int(cap), out, n,
                                          keep, int(n_threads), int(bool(dedup)))
    if rc != 0:
        raise MemoryError("oracle_run_batch_iterative failed")
    return out[:E], n[:E], keep[:x.size]


def max_threads() -> int:
    return int(lib().oracle_max_threads())
