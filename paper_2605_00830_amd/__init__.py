"""MI355X-native K-Best graph edit distance (FAST-GED method) library.

libged.so (HIP kernels for gfx950 behind the C ABI in include/ged.h) does
the work; paper_2605_00830_amd.ged is its Python binding and
paper_2605_00830_amd.synth draws seeded synthetic workloads.
"""
__version__ = "0.1.0"
