"""MI355X-native conformal Hough transform for drift-chamber hits.

The hot path (conformal map, theta sweep and voting, threshold + 3x3 peaks, retention mask)
runs in hand-written HIP kernels behind the C-ABI library libhough.so; `hough` is its thin
ctypes binding and `synth` the seeded synthetic event generator.  Importing the package does
not load the library; `paper_2607_04067_amd.hough` does, and fails loudly if it is not built.
"""
