"""Tile-size autotuner for the rasteriser.

Times one forward + backward of the actual problem (same Gaussians, same
keyframes) at tile sizes 8, 16 and 32 and keeps the fastest.  The LDS batch is
one splat record per lane of the tile's workgroup (64 records for 8x8 and
16x16 tiles, 256 for 32x32), so the tile size also fixes the batch.  Results
are cached per (Gaussian-count bucket, resolution multiset, SH degree,
checkpoint) for the life of the process.  Tile size changes which tiles a
splat is binned into, so parity is always checked at the chosen size.
"""
from __future__ import annotations

import math

import torch

from . import rasterizer as R

_cache = {}


def _key(params, cameras, checkpoint):
    res = tuple(sorted((c.width, c.height) for c in cameras))
    return (int(math.log2(max(params.n, 1))), res, params.sh_degree, bool(checkpoint))


def autotune_tile(params: R.GaussianParams, cameras, target, checkpoint=False, candidates=(8, 16, 32), iters=3):
    key = _key(params, cameras, checkpoint)
    if key in _cache:
        return _cache[key]
    from . import _lib as L
    times, skipped = {}, {}
    for tile in candidates:
        step = R.MappingStep(params, cameras, target, tile_size=tile, checkpoint=checkpoint, with_adam=False)
        try:
            step.size()
        except (L.GsError, torch.cuda.OutOfMemoryError) as e:  # pair count beyond the 32-bit index space / memory
            skipped[tile] = str(e).split("(")[-1].rstrip(")")
            del step
            torch.cuda.empty_cache()
            continue
        step.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            step.run()
        e1.record()
        torch.cuda.synchronize()
        times[tile] = round(e0.elapsed_time(e1) / iters, 4)
        del step
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    _cache[key] = {"best": best, "ms_fwd_bwd": times}
    if skipped:
        _cache[key]["skipped"] = skipped
    return _cache[key]
