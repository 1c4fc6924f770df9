"""MI355X-native spin-adapted DMRG hot path (arXiv:1312.2415, CheMPS2 method).

The compute lives in ``libsadmrg.so`` (HIP for gfx950, C ABI declared in
``include/sadmrg.h``); this package is a thin ctypes binding over it.
"""
from .binding import SaDMRG, load_library, library_path  # noqa: F401

__all__ = ["SaDMRG", "load_library", "library_path"]
