"""Device data-sharing runtime for generic-mode OpenMP-style target regions
on MI355X (gfx950): per-team frame stacks in LDS with an HBM overflow slab,
master-wave / worker-wave handoff, nested levels, exact reductions.

The compute path is libdsr.so (HIP); ``dsr`` is its ctypes binding.
"""
from . import dsr  # noqa: F401
