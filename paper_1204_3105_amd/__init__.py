"""MI355X (gfx950) hierarchical 2D FMM for the complex log kernel on the
square quadtree, septree and triangle-quadtree tilings.

The compute path is libfmm2d.so (HIP kernels behind the C ABI in
include/fmm2d.h); ``paper_1204_3105_amd.fmm`` is its Python binding.
"""
__all__ = ["fmm", "inputs"]
