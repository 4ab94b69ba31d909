"""ndrho: selected density-matrix elements by nested dissection and selected
inversion on an MI355X GPU (see include/ndrho.h for the C interface).

This module only marshals arguments into the C library libndrho.so; every
numerical step runs in the library's HIP kernels.  If the library has not been
built the import of the binding fails loudly (there is no fallback).
"""
from ._binding import (  # noqa: F401
    Context,
    DeviceBuffer,
    NdrhoError,
    Plan,
    cf_poles,
    lib_path,
    load_library,
    STATUS_NAMES,
)
