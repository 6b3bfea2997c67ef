"""MI355X-native hot path of the Parareal exponential-integrator Q1 FEM.

The compute lives in libpeifem.so (hand-written HIP for gfx950, C ABI in
include/peifem.h); ``peifem`` is its ctypes binding.  Importing this package
does not load the library; ``peifem.load_library()`` does, and raises when the
library has not been built.
"""
__all__ = ["peifem"]
