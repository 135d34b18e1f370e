"""MI355X (gfx950) mass-spring simulator: HIP kernels behind the C ABI in include/cronos.h.

``paper_2207_09334_amd.cronos`` is the ctypes binding (same entry-point names as the C ABI);
``paper_2207_09334_amd.problem`` turns a workload description into the arrays those entry
points take.  Build the native library with ``python -m paper_2207_09334_amd.build``.
"""
