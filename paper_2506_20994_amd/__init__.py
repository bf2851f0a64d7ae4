"""MI355X (gfx950) spectral-element operator library: Python binding.

Thin ctypes marshalling over libsem.so (include/sem.h).  Functions carry the
C names; tensors are torch tensors on the GPU, passed by data pointer, launched
on torch's current stream.  There is no CPU fallback: if libsem.so is missing
or fails to load, every entry point raises.
"""
from ._binding import *          # noqa: F401,F403
from ._binding import __all__    # noqa: F401
