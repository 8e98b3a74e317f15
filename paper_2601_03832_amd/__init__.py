"""Batched iterative Grover search on matrix product states, native to AMD MI355X (gfx950).

The compute path lives in ``csrc/`` (HIP kernels behind a C ABI declared in
``include/gmps.h``); :mod:`paper_2601_03832_amd.gmps` is the ctypes binding.
Importing this package does not load the shared library; the binding loads it
on first use and raises if it is missing.
"""

__all__ = ["inputs", "gmps"]
