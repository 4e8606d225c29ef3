"""MI355X (gfx950) differentiable Gaussian-splat rasterizer with the per-ray
entropy constraint on alpha-blending weights.

`gsr` is the binding of the HIP library libgsr.so (include/gsr.h); `scenes`
draws seeded synthetic inputs.  Build the library with `build.build()`.
"""
__all__ = ["gsr", "scenes", "build"]
