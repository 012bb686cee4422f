"""Host-only checks of the C-ABI library: it loads and exports what include/hough.h declares.

No compute call is made here (there is no GPU in this environment)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_04067_amd", "libhough.so")


@pytest.fixture(scope="module")
def hough_mod():
    if not os.path.exists(LIB):
        from paper_2607_04067_amd import build
        build.build()
    from paper_2607_04067_amd import hough
    return hough


def test_library_exports_every_declared_function(hough_mod):
    lib = hough_mod.load()
    names = hough_mod.header_functions()
    assert {"hough_config", "hough_vote", "hough_peaks", "hough_retain", "hough_run_batch"} <= set(names)
    serve = hough_mod.header_functions(os.path.join(ROOT, "include", "hough_serve.h"))
    assert serve == ["hough_serve_run", "hough_serve_simulate"]
    for n in names + serve:
        assert hasattr(lib, n), n


def test_struct_layouts_match_header(hough_mod):
    text = open(os.path.join(ROOT, "include", "hough.h")).read()
    # hough_params: 2 x int32, 2 x double, 6 x int32 = 48 bytes; hough_peak: 8 bytes
    assert ctypes.sizeof(hough_mod.hough_params) == 48
    params = re.sub(r"/\*.*?\*/", "", re.search(r"typedef struct hough_params \{(.*?)\}", text, re.S).group(1),
                    flags=re.S)
    assert re.findall(r"\b(?:int32_t|double)\s+(\w+)", params) == [n for n, _ in hough_mod.hough_params._fields_]
    peak = re.search(r"typedef struct hough_peak \{(.*?)\}", text, re.S).group(1)
    assert re.findall(r"(uint\d+_t)", peak) == ["uint16_t", "uint16_t", "uint32_t"]
    # hough_track: five doubles, int32 charge, uint32 n_hits = 48 bytes, as decode_tracks reads it
    track = re.sub(r"/\*.*?\*/", "", re.search(r"typedef struct hough_track \{(.*?)\}", text, re.S).group(1),
                   flags=re.S)
    assert re.findall(r"\b(double|int32_t|uint32_t)\b", track) == ["double"] * 4 + ["int32_t", "uint32_t"]
    assert track.count(",") == 1 and hough_mod.TRACK_DTYPE.itemsize == 48
    assert hough_mod.TRACK_DTYPE.names == ("a", "b", "radius", "pt", "phi_c", "charge", "n_hits")


def test_serve_config_layout_matches_header():
    from paper_2607_04067_amd import serve
    text = open(os.path.join(ROOT, "include", "hough_serve.h")).read()
    body = re.sub(r"/\*.*?\*/", "", re.search(r"typedef struct hough_serve_config \{(.*?)\}", text, re.S).group(1),
                  flags=re.S)
    fields = re.findall(r"\b(int32_t|double)\s+(\w+);", body)
    assert [n for _, n in fields] == [n for n, _ in serve.hough_serve_config._fields_]
    assert ctypes.sizeof(serve.hough_serve_config) == 40


def test_status_strings(hough_mod):
    for code in (0, -1, -2, -3, -4, -5):
        assert hough_mod.status_string(code) != "unknown status"
    assert hough_mod.status_string(-6) == "unknown status"


def test_config_reports_enomem_when_allocation_fails(hough_mod, monkeypatch):
    """hough_config's allocation-failure path: with HOUGH_TEST_FAIL_ALLOC=1 a valid grid gets
    HOUGH_ENOMEM and no context, before any device call (so this runs without a GPU).  Invalid
    grids are still refused as HOUGH_EINVAL first."""
    lib = hough_mod.load()
    p = hough_mod.hough_params(360, 256, -0.005, 0.005, hough_mod.ACC_I32, 10, 1, 64, 0, 0)
    bad = hough_mod.hough_params(360, 0, -0.005, 0.005, hough_mod.ACC_I32, 10, 1, 64, 0, 0)
    ctx = ctypes.c_void_p(12345)
    monkeypatch.setenv("HOUGH_TEST_FAIL_ALLOC", "1")
    assert lib.hough_config(ctypes.byref(p), ctypes.byref(ctx)) == hough_mod.HOUGH_ENOMEM
    assert not ctx.value
    assert lib.hough_config(ctypes.byref(bad), ctypes.byref(ctx)) == hough_mod.HOUGH_EINVAL
    assert lib.hough_config(None, ctypes.byref(ctx)) == hough_mod.HOUGH_EINVAL
    lib.hough_destroy(None)                       # destroying nothing is a no-op


def test_static_scratch_limit_matches_header(hough_mod):
    text = open(os.path.join(ROOT, "include", "hough.h")).read()
    m = re.search(r"#define HOUGH_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == hough_mod.STATIC_SCRATCH_BYTES
    assert re.search(r"#define HOUGH_ETOOLARGE \(-5\)", text) and hough_mod.HOUGH_ETOOLARGE == -5


def test_phase_timing_build_exports_its_hook_and_the_product_does_not(hough_mod):
    """The instrumented build (libhough_phases.so) exports hough_debug_phase_ticks beside every
    product function; libhough.so does not export it."""
    from paper_2607_04067_amd import build
    if not os.path.exists(build.PHASES_LIB):
        build.build_phases()
    phases = ctypes.CDLL(build.PHASES_LIB)
    dbg = hough_mod.header_functions(os.path.join(ROOT, "include", "hough_debug.h"))
    assert dbg == ["hough_debug_phase_ticks"]
    for n in hough_mod.header_functions() + dbg:
        assert hasattr(phases, n), n
    assert not hasattr(hough_mod.load(), "hough_debug_phase_ticks")


def test_peak_record_decoding(hough_mod):
    import numpy as np
    rec = np.array([[3 | (17 << 16), 42], [65535 | (1 << 16), 7]], dtype=np.uint32).view(np.int32)
    assert hough_mod.decode_peaks(rec).tolist() == [[3, 17, 42], [65535, 1, 7]]


def test_product_path_never_touches_the_oracle():
    """Nothing under the package may import, load or run the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2607_04067_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                for pat in (r"import\s+oracle", r"from\s+oracle", r"liboracle", r"hough_oracle",
                            r"oracle_[a-z]+\s*\("):
                    assert not re.search(pat, text), (f, pat)
