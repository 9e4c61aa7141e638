"""Matrix-free NGF + curvature image registration on MI355X (gfx950).

The computation lives in the HIP library ``_lib/libmfr.so`` (C ABI declared in
``include/mfr.h``); ``paper_1804_10541_amd.mfr`` is its ctypes binding.
Importing the package does not load the library; ``mfr.load()`` (called by
every binding entry point) raises if it is missing.
"""
__all__ = ["mfr"]
