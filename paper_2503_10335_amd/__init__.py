"""MI355X-native TPB sigma build (H*C), Davidson solver and serving loop.

The compute path is the C-ABI library ``libtbsci.so`` (HIP kernels for
gfx950) declared in ``include/tbsci.h``; ``paper_2503_10335_amd.tbsci`` is
its thin ctypes binding.  ``workloads`` draws seeded synthetic inputs.
"""
__all__ = ["workloads", "tbsci"]
