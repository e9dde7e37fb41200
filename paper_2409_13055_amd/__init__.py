"""MI355X (gfx950) implementation of the mapping hot path of MGSO (arxiv 2409.13055):
the tile-based differentiable 3D Gaussian splatting rasteriser and its Adam step,
behind the C ABI of include/gs.h.

Submodules are imported lazily: `synthetic` (seeded workloads) needs no GPU;
`rasterizer` and `_lib` load libgs.so and fail loudly when it is missing.
"""
__all__ = ["synthetic", "rasterizer"]
