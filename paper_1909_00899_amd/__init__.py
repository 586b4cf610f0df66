"""MI355X striped-scan Smith-Waterman (affine gaps, Gotoh) behind a C ABI.

The compute path is hand-written HIP for gfx950 in ``csrc/``, built into
``libswscan.so``; ``api`` is a thin ctypes binding with the same entry-point
names.  The native library is loaded lazily on first use and a missing or
unloadable library raises: there is no CPU fallback.
"""
from . import workloads  # noqa: F401  (input generators only; no alignment arithmetic)

__all__ = ["workloads"]
