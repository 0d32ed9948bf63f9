"""MI355X-native page-cipher engine for MemShield's GPU hot path.

The compute path lives in ``libmemshield.so`` (HIP kernels for gfx950 behind
a C ABI declared in ``include/memshield.h``); ``memshield`` is its thin
ctypes binding.  Importing this package loads nothing; the library is loaded
on first use by ``paper_2004_09252_amd.memshield`` and a missing library is
an error, never a fallback.
"""
__all__ = ["memshield", "workloads"]
