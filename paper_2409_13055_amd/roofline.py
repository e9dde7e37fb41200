"""Algorithmic work of each hot-path call, for roofline reporting.

Bytes are what the method must move through HBM: each input read once and
each output written once (not the implementation's extra passes or cache
re-reads).  For the raster calls the arithmetic is counted too, as FP32
flops of the (pixel, entry) pairs that blend (counted exactly on the GPU by
gs_render_stats), because those kernels are bound by vector ALU issue, not
by HBM.

Per-unit figures (P_n = 11 + 3K raw floats per Gaussian, K = (D+1)^2):
  project     N*4*P_n + V*N*4 [tiles_touched] + Nv*(48 + 16) [visible records and entries] + S*4 [segment counts]
  bin_sort    S*4 [segment counts] + Nv*16 [visible-pair entries] + L [the lists]
  render_fwd  Nv*36 + L + Px*(12 + 12 [target] + 8 [T_final, n_contrib unless checkpoint])
  raster_bwd  Px*(12 [image] + 12 [target]) + Nv*36 [records] + L + Nv*36 [gradients]
  project_bwd N*(4*P_n + 8*P_n) + V*N*(36 + 16)
  render_bwd  raster_bwd + project_bwd
  adam        N*P_n*32  (read p, g, m, v; write p, m, v, g := 0)
  project_bwd_adam  N*P_n*24 (read p, m, v; write p, m, v) + V*N*52
with N Gaussians, V views, Nv visible (view, Gaussian) pairs, S = V*ceil(N/64)
projection segments, Px pixels, and L the bytes of the bins: M*4 [ids] + T*8
[ranges] for tile lists (M incidences, T tiles), E*8 [items] + W*8 [window
ranges] for window lists (E items, W windows).
"""
from __future__ import annotations

import torch

# FP32 operations of the per-pixel blending (an FMA counts 2; a compare, min,
# exp2 or reciprocal counts 1), per (pixel, list entry):
#   evaluated entry  17: d = pixel - mean 2; power 9 (3 mul, 2 FMA, 1 scale);
#                        power > 0 test 1; exp 2; opacity * G 1; min 1;
#                        alpha test 1
#   blended, forward +10: 1 - alpha, T (1 - alpha), T test, weight, colour 3 FMA
#   blended, backward +44: 1 - alpha, T (1 - alpha), T test, weight, colour
#                        behind (3 FMA), colour grads (3 FMA), dL/dC . c and
#                        dL/dC . S (mul + 2 FMA each), reciprocal, dL/dalpha
#                        (mul + FMA), clamp test, dL/dpower, opacity grad FMA,
#                        u dx and u dy, moments (2 add + 3 FMA)
# Only the blended pairs are counted, each with its evaluation: an evaluation
# that does not blend is work a cull can avoid (the kernels skip most of them),
# so counting it would credit work that is not done.  The counts come from
# gs_render_stats (the blending as defined): E_blend blended pairs; E_eval,
# the entries evaluated until each pixel stops, is reported beside it.
FLOPS_EVAL = 17
FLOPS_FWD_BLEND = 10
FLOPS_BWD_BLEND = 44


def counts(step, sc):
    fr = step.frame
    n, V = step.params.n, step.rast.n_views
    K = (step.params.sh_degree + 1) ** 2
    pn = 11 + 3 * K
    win = bool(getattr(fr, "windowed", False))
    return dict(N=n, V=V, Pn=pn, M=int(fr.d_num_pairs.item()), Nv=int(torch.count_nonzero(fr.tiles).item()),
                Px=step.rast.total_pixels, T=step.rast.total_tiles, ckpt=step.rast.checkpoint, windowed=win,
                E=int(fr.d_num_items.item()) if win else 0, W=step.rast.total_windows if win else 0)


def algorithmic_bytes(c):
    N, V, Pn, M, Nv, Px, T = c["N"], c["V"], c["Pn"], c["M"], c["Nv"], c["Px"], c["T"]
    S = V * ((N + 63) // 64)
    saved = 0 if c["ckpt"] else 8
    lists = c["E"] * 8 + c["W"] * 8 if c.get("windowed") else M * 4 + T * 8
    raster_bwd = Px * 24 + Nv * 36 + lists + Nv * 36
    project_bwd = N * 12 * Pn + V * N * 52
    return {
        "project": N * 4 * Pn + V * N * 4 + Nv * (48 + 16) + S * 4,
        "bin_sort": S * 4 + Nv * 16 + lists,
        "render_fwd": Nv * 36 + lists + Px * (24 + saved),
        "raster_bwd": raster_bwd,
        "project_bwd": project_bwd,
        "render_bwd": raster_bwd + project_bwd,
        "adam": N * Pn * 32,
        "project_bwd_adam": N * 24 * Pn + V * N * 52,
    }


def evaluations(step):
    """Exact work counts of the blending of the step's frame (gs_render_stats)."""
    return step.rast.render_stats(step.frame)


def alu_flops(kernel, ev):
    blend = FLOPS_FWD_BLEND if kernel == "render_fwd" else FLOPS_BWD_BLEND
    return ev["blended"] * (FLOPS_EVAL + blend)


SINGLE_KERNEL_CALLS = ("project", "render_fwd", "raster_bwd", "project_bwd", "adam", "project_bwd_adam")


def step_bytes(b, stages):
    """Algorithmic bytes of one iteration made of the given single-call stages."""
    return sum(b[k] for k in stages if k in b)


def report(step, sc, stages_ms, hbm_peak_gbs, valu_peak_tflops, valu_unpacked_tflops, traffic=None, work=None,
           step_ms=None):
    """Roofline of the dominant single-kernel call (by measured duration), and of the whole step.
    `work`: blending work counts averaged over the timed iterations (default: counted on the step's
    current lists).  The raster calls are priced against FP32 vector issue, both at the published
    peak (which needs packed FP32 instructions) and at the rate without them; their HBM bytes are
    listed but given no bandwidth fraction, since they stop reading a tile's list where its pixels
    terminate.  `step_ms`: the measured time of the whole iteration (graph replay)."""
    c = counts(step, sc)
    b = algorithmic_bytes(c)
    ev = work if work is not None else evaluations(step)
    dom = max((k for k in stages_ms if k in SINGLE_KERNEL_CALLS), key=lambda k: stages_ms[k])
    ms = stages_ms[dom]
    per_stage = {}
    for k in stages_ms:
        if k not in b:
            continue
        e = {"ms": stages_ms[k], "alg_bytes": b[k]}
        if k in ("render_fwd", "raster_bwd"):
            e["TFLOPs"] = round(alu_flops(k, ev) / (stages_ms[k] * 1e-3) / 1e12, 3)
        else:
            e["GBps"] = round(b[k] / (stages_ms[k] * 1e-3) / 1e9, 1)
            e["hbm_frac"] = round(e["GBps"] / hbm_peak_gbs, 4)
        per_stage[k] = e
    if dom in ("render_fwd", "raster_bwd"):
        flops = alu_flops(dom, ev)
        achieved = flops / (ms * 1e-3) / 1e12
        out = {"bound": "alu", "achieved": round(achieved, 3), "peak": valu_peak_tflops, "unit": "TFLOP/s",
               "frac": round(achieved / valu_peak_tflops, 4), "traffic": traffic, "kernel": dom,
               "peak_without_packed_fp32": valu_unpacked_tflops,
               "frac_without_packed_fp32": round(achieved / valu_unpacked_tflops, 4),
               "flops_per_launch": flops, "evaluations": ev, "ms_per_launch": ms}
    else:
        achieved = b[dom] / (ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": hbm_peak_gbs, "unit": "GB/s",
               "frac": round(achieved / hbm_peak_gbs, 4), "traffic": traffic, "kernel": dom,
               "alg_bytes_per_launch": b[dom], "ms_per_launch": ms}
    stages = [k for k in stages_ms if k in SINGLE_KERNEL_CALLS or k == "bin_sort"]
    alg = step_bytes(b, stages)
    t = step_ms if step_ms is not None else stages_ms.get("step_eager")
    gbs = alg / (t * 1e-3) / 1e9
    out["step"] = {"stages": stages, "alg_bytes": alg, "ms": round(t, 4), "GBps": round(gbs, 1),
                   "hbm_frac": round(gbs / hbm_peak_gbs, 4)}
    out["stages"] = per_stage
    out["counts"] = c
    return out
