"""Tile-size autotuning through the library's gs_autotune (include/gs.h).

gs_autotune times one iteration of the actual problem (projection, bin/sort,
forward with the L1 term, raster backward, projection backward) at tile sizes
8, 16 and 32 on the current stream and keeps the fastest; the LDS batch is one
splat record per lane of the tile's workgroup, so the tile size also fixes it.
The library caches the result per (Gaussian-count bucket, resolution
multiset, SH degree, checkpoint) for the life of the process.  Tile size
changes which tiles a splat is binned into, so parity is always checked at the
chosen size.  This module only marshals the arguments.
"""
from __future__ import annotations

import torch

from . import _lib as L
from . import rasterizer as R

_TILES = (8, 16, 32)


def autotune_tile(params: R.GaussianParams, cameras, target: torch.Tensor, checkpoint=False, candidates=_TILES,
                  iters=3, refresh=False):
    """Returns {"best": tile, "ms_fwd_bwd": {tile: ms}, "pairs": {tile: M}, "from_cache": bool}
    (ms -1 for a candidate that did not fit in device memory)."""
    L.load()
    cams = L.make_cameras(list(cameras))
    opts = L.default_options(checkpoint=int(checkpoint))
    mask = sum(1 << _TILES.index(int(t)) for t in candidates)
    torch.cuda.synchronize()
    r = L.gs_autotune(params.c_params(), cams, len(cameras), opts, target.data_ptr(), int(iters), mask,
                      1 if refresh else 0, torch.cuda.current_stream().cuda_stream)
    tiles = [r.candidates[k] for k in range(r.n_candidates)]
    return {"best": int(r.tile_size), "ms_fwd_bwd": {t: round(float(r.ms[k]), 4) for k, t in enumerate(tiles)},
            "pairs": {t: int(r.pairs[k]) for k, t in enumerate(tiles)}, "from_cache": bool(r.from_cache)}
