"""Banded Smith-Waterman seed extension (BSW) on AMD Instinct MI355X.

``paper_1907_12931_amd.bsw`` is the ctypes binding of ``libbsw.so`` (HIP
kernels for gfx950 behind a C ABI); ``synth`` draws seeded workloads.
Importing the package loads nothing; the library is loaded on first use.
"""
