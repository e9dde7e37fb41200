"""Autotuning through the library's gs_autotune (include/gs.h).

gs_autotune times one iteration of the actual problem (projection, bin/sort,
forward with the L1 term, raster backward, projection backward) for every
candidate tile size (8, 16, 32), LDS batch of the raster kernels (one or two
splat records per lane) and form of the bins (tile lists or window lists) on
the current stream and keeps the fastest.  The library caches the result per
(Gaussian-count bucket, resolution multiset, SH degree, checkpoint, other
option flags, candidates) for the life of the process.  Tile size changes
which tiles a splat is binned into, so parity is always checked at the chosen
size; the LDS batch and the bins form change no output.  This module only
marshals the arguments.
"""
from __future__ import annotations

import torch

from . import _lib as L
from . import rasterizer as R

_TILES = (8, 16, 32)
_BATCHES = (1, 2)


def autotune_tile(params: R.GaussianParams, cameras, target: torch.Tensor, checkpoint=False, candidates=_TILES,
                  batches=_BATCHES, iters=3, refresh=False, lists="auto"):
    """Returns {"best": tile, "lds_batch": b, "lists": "window" or "tile", "ms_fwd_bwd":
    {"tile/batch/lists": ms}, "pairs": {tile: M}, "from_cache": bool} (ms -1 for a candidate that did
    not fit in device memory).  lists: "auto" times both forms of the bins, else only the one named."""
    L.load()
    if lists not in ("auto", "window", "tile"):
        raise ValueError(f"lists must be 'auto', 'window' or 'tile', not {lists!r}")
    cams = L.make_cameras(list(cameras))
    opts = L.default_options(checkpoint=int(checkpoint))
    forms = {"auto": 0, "tile": 1 << 5, "window": 1 << 6}[lists]
    mask = sum(1 << _TILES.index(int(t)) for t in candidates) | \
        sum(1 << (3 + _BATCHES.index(int(b))) for b in batches) | forms
    torch.cuda.synchronize()
    r = L.gs_autotune(params.c_params(), cams, len(cameras), opts, target.data_ptr(), int(iters), mask,
                      1 if refresh else 0, torch.cuda.current_stream().cuda_stream)
    k_all = range(r.n_candidates)
    name = ("tile", "window")
    return {"best": int(r.tile_size), "lds_batch": int(r.lds_batch), "lists": name[int(r.window_lists)],
            "ms_fwd_bwd": {f"{r.cand_tile[k]}/{r.cand_batch[k]}/{name[r.cand_window[k]]}": round(float(r.ms[k]), 4)
                           for k in k_all},
            "pairs": {int(r.cand_tile[k]): int(r.pairs[k]) for k in k_all}, "from_cache": bool(r.from_cache)}
