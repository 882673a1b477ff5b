"""MI355X-native surfel feature rasterizer (the rendering path of Fast-SegSim,
arXiv 2604.10951): preprocess, precise tile intersection, key sort and
front-to-back blending of C-channel features, full or with Top-K hard
selection, plus its backward, as hand-written HIP kernels for gfx950 behind a
C ABI (include/fastsegsim.h).

Importing the package does not load the HIP library; ``raster.Rasterizer``
does, and fails loudly if it has not been built.
"""
from . import scenes  # noqa: F401

__all__ = ["scenes", "raster", "build"]
