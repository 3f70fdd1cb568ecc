"""Relaxed-order FMM-BEM solves on AMD Instinct MI355X (gfx950).

The compute path lives in libfmmbem.so (hand-written HIP, C ABI declared in
include/fmmbem.h); `paper_1506_05957_amd.fmmbem` is its thin ctypes binding.
Importing this package does not load the library; `fmmbem` does, and fails
loudly when the library has not been built.
"""
