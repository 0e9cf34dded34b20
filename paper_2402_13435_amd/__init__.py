"""Exhaustive filtered top-K retrieval on AMD MI355X (gfx950).

A C-ABI library of hand-written HIP kernels (``include/fr.h``,
``csrc/``) with a thin ctypes binding.  See ``binding.Index``.
"""
from .binding import (Cnf, FrError, Index, SearchResult, lib,  # noqa: F401
                      FR_DEVICE_PTRS, FR_GRAPH, FR_NOWAIT, STATUS_NAMES, SYMBOLS)
