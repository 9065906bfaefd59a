"""Tiled composite SpMV for power-law graph matrices on MI355X (gfx950).

The compute path is the HIP library libtcspmv.so (C ABI in include/tcspmv.h);
`tc` is its Python binding.  Importing this package does not load the library;
the first call does, and raises if it is not built.
"""
from .tc import (DeviceCsr, NotConverged, TcError, TiledMatrix, build_tiled, csr_spmv,  # noqa: F401
                 load_library, release_cached_memory, rwr_multi)
