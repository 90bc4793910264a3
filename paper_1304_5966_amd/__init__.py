"""Exact affine-gap Smith-Waterman (SW#-style score, start and Myers-Miller
reconstruction) on AMD Instinct MI355X (gfx950).

The compute lives in ``libswmi.so`` (hand-written HIP kernels behind a C ABI,
declared in ``include/swmi.h``); ``paper_1304_5966_amd.swmi`` is the thin
ctypes binding.  ``paper_1304_5966_amd.synth`` generates the seeded synthetic
workloads.  Importing the package loads nothing.
"""
