"""MI355X (gfx950) spectral canonical electrostatic library: Python binding.

A thin ctypes layer over the C ABI in ``include/sce.h`` (``libsce.so``, built
by ``paper_1508_07344_amd.build``).  Every computation runs in the library's
HIP kernels; this module only marshals arguments.  torch tensors provide
device memory and streams.  There is no CPU fallback: if the library is not
built, or no GPU is visible, calls raise.
"""
from .sce import (SCE_OK, SCE_EINVAL, SCE_ENOMEM, SCE_EDEVICE, SCE_ESTATE, SCE_ENOTSUP,
                  SCE_EUNSTABLE, PREC, SCHEME, SHAPE, Diag, SceError, Context, Server, load_library,
                  library_path, exported_symbols)

__all__ = ["SCE_OK", "SCE_EINVAL", "SCE_ENOMEM", "SCE_EDEVICE", "SCE_ESTATE", "SCE_ENOTSUP",
           "SCE_EUNSTABLE", "PREC", "SCHEME", "SHAPE", "Diag", "SceError", "Context", "Server",
           "load_library", "library_path", "exported_symbols"]
