"""MI355X-native brick-based Gaussian-to-voxel rasterizer (normalised aggregation) and its gradient.

The GPU library is ``libgs.so`` (HIP for gfx950, C ABI declared in ``include/gs.h``); ``gs`` is its
thin Python binding.  Importing this package loads nothing; ``from paper_2603_09621_amd import gs``
loads the library and fails loudly when it is missing.
"""
__all__ = ["gs", "synth"]
