"""MI355X implementation of the directional scale-discretized wavelet transform
on the sphere (analysis, exact synthesis, scaling coefficients).

The transforms run in hand-written HIP kernels behind the C ABI declared in
``include/s2dw.h``; ``paper_1308_5706_amd.s2dw`` is the thin Python binding.
"""
__all__ = ["inputs", "s2dw"]
