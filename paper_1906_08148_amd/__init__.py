"""MI355X (gfx950) library for approximate products of matrices with decay:
Truncmul, SpAMM and Hybrid on quadtrees of dense leaf blocks (arXiv:1906.08148).

The compute path is the HIP library ``_lib/libspamm.so`` (C-ABI in
``include/spamm.h``); ``spamm`` is its ctypes binding.  Importing this package
does not load the library; ``spamm.load_library()`` or creating a
``spamm.Context`` does, and raises when the library is missing.
"""
__all__ = ["spamm"]
