"""MI355X-native condensed-history proton transport Monte Carlo with dose
scoring (after Wan Chan Tseung, Ma & Beltran, arXiv:1409.8336).

The transport runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/pmc.h``; :mod:`paper_1409_8336_amd.pmc` is the thin ctypes
binding and :mod:`paper_1409_8336_amd.synth` the seeded input generators.
"""
