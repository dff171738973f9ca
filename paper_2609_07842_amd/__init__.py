"""MI355X-native hot path of the valency-bounding correction (VBC), arXiv 2609.07842.

The compute path is the HIP library ``libvbc.so`` (kernels for gfx950 behind a
C ABI declared in ``include/vbc.h``); ``paper_2609_07842_amd.vbc`` is a thin
ctypes binding with the same entry-point names.  Importing this package does not
load the library; ``paper_2609_07842_amd.vbc`` does, and fails loudly if it has
not been built.
"""
__all__ = ["workloads"]
