"""MI355X-native separated-operator apply on Legendre multiwavelet octrees.

The computation lives in libmra.so (C ABI in include/mra.h): host planning in C++ and
HIP kernels for gfx950.  This package only marshals arguments; it raises ImportError-like
errors when the library is missing instead of falling back to anything else.
"""
from ._binding import (Context, Function, Operator, MraError, load, host_fit, host_block,
                       host_filters, host_spectral_norm, host_project, EXPORTED, LIB_PATH,
                       REPR_SCALING, REPR_WAVELET)

__all__ = ["Context", "Function", "Operator", "MraError", "load", "host_fit", "host_block",
           "host_filters", "host_spectral_norm", "host_project", "EXPORTED", "LIB_PATH",
           "REPR_SCALING", "REPR_WAVELET"]
