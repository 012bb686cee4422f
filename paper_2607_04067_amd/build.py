"""Build the package's HIP libraries (gfx950) in-tree with hipcc.

libhough.so        the C ABI of include/hough.h and include/hough_serve.h (the product);
libhough_probe.so  a measurement probe (the LDS atomic rate of the vote's access pattern);
libhough_phases.so the product sources compiled with HOUGH_PHASE_TIMING: the fused kernel
                   also times its phases (include/hough_debug.h).  Measurement only.

Flags that matter for exactness: -ffp-contract=off (only the explicit fmaf calls fuse),
correctly rounded single-precision division, denormals kept (no flush-to-zero) and no
fast-math.  Packed FP32 instructions are disabled (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhough.so")
SOURCES = ["hough_kernels.hip", "hough_scratch.hip", "hough_api.cpp", "hough_serve.cpp"]
PROBE_LIB = os.path.join(HERE, "libhough_probe.so")
PROBE_SOURCES = ["hough_probe.hip"]
ARCH = os.environ.get("HOUGH_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero", "-fno-gpu-rdc",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(sources, out: str, extra=(), verbose: bool = False) -> str:
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, *[os.path.join(CSRC, s) for s in sources], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(out: str = LIB, verbose: bool = False) -> str:
    """Compile the product library into `out` (always recompiles)."""
    return _compile(SOURCES, out, verbose=verbose)


def build_probe(out: str = PROBE_LIB, verbose: bool = False) -> str:
    """Compile the measurement probe library (always recompiles)."""
    return _compile(PROBE_SOURCES, out, verbose=verbose)


PHASES_LIB = os.path.join(HERE, "libhough_phases.so")


def build_phases(out: str = PHASES_LIB, verbose: bool = False) -> str:
    """Compile the phase-timing build of the product sources (always recompiles)."""
    return _compile(SOURCES, out, extra=("-DHOUGH_PHASE_TIMING",), verbose=verbose)


def build_all(verbose: bool = False) -> list[str]:
    return [build(verbose=verbose), build_probe(verbose=verbose), build_phases(verbose=verbose)]


if __name__ == "__main__":
    print(build_all(verbose="-v" in sys.argv))
