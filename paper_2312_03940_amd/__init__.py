"""MI355X-native DPC hot path of PECANN (arXiv 2312.03940).

The compute path is ``libpecann.so`` (hand-written HIP kernels for gfx950 behind a
C ABI, declared in ``include/pecann.h``); ``paper_2312_03940_amd.pecann`` is its thin
ctypes binding.  Nothing is loaded at import time, so importing the package (or its
``datagen`` module) never touches a GPU.
"""
__all__ = ["datagen", "pecann"]
