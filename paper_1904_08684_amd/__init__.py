"""MI355X-native geometric-multigrid V-cycle (HIP kernels for gfx950 behind a C ABI).

Importing the package loads nothing; ``paper_1904_08684_amd.mg`` is the
binding to the HIP library and ``paper_1904_08684_amd.workloads`` holds the
seeded input generators.
"""
__version__ = "0.1.0"
