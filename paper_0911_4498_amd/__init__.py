"""MI355X (gfx950) implementation of fast Basic SSA.

The compute path lives in the HIP shared library built from ``csrc/``; the
Python module :mod:`paper_0911_4498_amd.ssa` is a thin ctypes binding over
its C ABI (``include/ssa.h``).  Importing this package loads nothing.
"""
