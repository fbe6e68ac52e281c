"""Continuous-scale central-moment lattice Boltzmann on AMD MI355X (gfx950).

The compute path is ``libcslbm.so`` (hand-written HIP kernels behind the C ABI
declared in ``include/cslbm.h``).  ``level.Level`` drives it with torch-owned
device buffers; ``inputs`` holds the seeded synthetic workloads.
"""
