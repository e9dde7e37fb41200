"""Algorithmic work of each hot-path call, for roofline reporting.

Bytes are what the method must move through HBM: each input read once and
each output written once (not the implementation's extra passes or cache
re-reads).  For the raster calls the arithmetic is counted too, as FP32
flops per (pixel, splat) evaluation times a lower bound on the evaluations
(sum over pixels of the number of list entries up to the last blended one),
because those kernels are bound by vector ALU issue, not by HBM.

Per-unit figures (P_n = 11 + 3K raw floats per Gaussian, K = (D+1)^2):
  project     N*4*P_n + V*N*(48 + 4)
  bin_sort    V*N*8 + M*(12 + 24 + 8) + T*8
  render_fwd  Nv*36 + M*4 + Px*(12 + 12 [target] + 8 [T_final, n_contrib unless checkpoint])
  render_bwd  Px*(12 + 12 + 8 [unless checkpoint]) + Nv*36 + M*4 + V*N*36
              + N*(4*P_n + 8*P_n) + V*N*(36 + 16)
  adam        N*P_n*32  (read p, g, m, v; write p, m, v, g := 0)
with N Gaussians, V views, Nv visible (view, Gaussian) pairs, M tile
incidences, Px pixels and T tiles.
"""
from __future__ import annotations

import torch

FLOPS_FWD_EVAL = 26   # dx,dy 2; power 10; exp 2; alpha 3; T test 3; weight 1; colour 6 (FMA = 2)
FLOPS_BWD_EVAL = 66   # recompute 18; T 3; colour grads 7; dL/dalpha 15; S update 6; opacity/power 3; mean/conic 14


def counts(step, sc):
    fr = step.frame
    n, V = step.params.n, step.rast.n_views
    K = (step.params.sh_degree + 1) ** 2
    pn = 11 + 3 * K
    return dict(N=n, V=V, Pn=pn, M=int(fr.d_num_pairs.item()), Nv=int(torch.count_nonzero(fr.tiles).item()),
                Px=step.rast.total_pixels, T=step.rast.total_tiles, ckpt=step.rast.checkpoint)


def algorithmic_bytes(c):
    N, V, Pn, M, Nv, Px, T = c["N"], c["V"], c["Pn"], c["M"], c["Nv"], c["Px"], c["T"]
    saved = 0 if c["ckpt"] else 8
    return {
        "project": N * 4 * Pn + V * N * 52,
        "bin_sort": V * N * 8 + M * 44 + T * 8,
        "render_fwd": Nv * 36 + M * 4 + Px * (24 + saved),
        "render_bwd": Px * (24 + saved) + Nv * 36 + M * 4 + V * N * 36 + N * 12 * Pn + V * N * 52,
        "adam": N * Pn * 32,
    }


def evaluations(step):
    """Lower bound on (pixel, splat) evaluations: sum of contributor counts of a forward render."""
    from . import rasterizer as R
    r = step.rast
    if not r.checkpoint:
        fr = step.frame
        r.render_fwd(fr)
        return int(fr.n_contrib.to(torch.int64).sum().item())
    probe = R.Rasterizer(r.cameras, r.n, r.sh_degree, tile_size=r.opts.tile_size, checkpoint=False,
                         device=r.device)
    probe.reserve(r.capacity)
    fr = probe.forward(step.params)
    e = int(fr.n_contrib.to(torch.int64).sum().item())
    del fr, probe
    return e


def report(step, sc, stages_ms, hbm_peak_gbs, valu_peak_tops):
    c = counts(step, sc)
    b = algorithmic_bytes(c)
    ev = evaluations(step)
    dom = max((k for k in stages_ms if k in b), key=lambda k: stages_ms[k])
    ms = stages_ms[dom]
    per_stage = {k: {"ms": stages_ms[k], "alg_bytes": b[k], "GBps": round(b[k] / (stages_ms[k] * 1e-3) / 1e9, 1)}
                 for k in stages_ms if k in b}
    if dom in ("render_fwd", "render_bwd"):
        flops = ev * (FLOPS_FWD_EVAL if dom == "render_fwd" else FLOPS_BWD_EVAL)
        achieved = flops / (ms * 1e-3) / 1e12
        peak = 2 * valu_peak_tops  # FMA counted as 2 flops, no packed FP32
        out = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2), "unit": "TFLOP/s",
               "frac": round(achieved / peak, 4), "traffic": None, "kernel": dom, "evaluations": ev}
    else:
        achieved = b[dom] / (ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": hbm_peak_gbs, "unit": "GB/s",
               "frac": round(achieved / hbm_peak_gbs, 4), "traffic": None, "kernel": dom}
    out["stages"] = per_stage
    out["counts"] = c
    return out
