"""Benchmark of the mapping step: Mpix*iter/s on one MI355X, batched vs per-view.

A step is one mapping iteration over the workload's keyframes: projection,
tile binning/sort, forward with the fused L1 loss, backward, and Adam when the
workload includes it.  The batched path replays one HIP graph per step; the
per-view path launches the same kernels view by view (no graph).  Inputs are
seeded synthetic scenes already resident in HBM when timing starts.

Prints one JSON line (see the keys below).  Default workload: 2M Gaussians,
16 keyframes at 1200x680, SH degree 3, fwd+bwd+Adam, transmittance recomputed
in the backward (checkpoint).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
# FP32 vector peak: 256 CU * 4 SIMD * 16 lanes * 2 flop (FMA) * 2 (packed FP32) * 2.4 GHz = 157.3
# TFLOP/s published; the build disables packed-FP32 instructions, which halves the rate it can reach.
VALU_PEAK_TFLOPS = 157.29
VALU_UNPACKED_TFLOPS = 78.64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=5, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--tile", type=int, default=0, help="tile size (0: autotune over 8/16/32)")
    ap.add_argument("--lds-batch", type=int, default=0, choices=[0, 1, 2],
                    help="splat records per lane per LDS batch (0: autotuned with the tile, or 1 at a fixed tile)")
    ap.add_argument("--layout", default="morton", choices=["morton", "generated"],
                    help="order of the Gaussian set in memory: Morton order of the means (gs_spatial_order, the "
                         "layout the mapping loop keeps) or the order the scene generator drew them in")
    ap.add_argument("--lists", default="auto", choices=["auto", "window", "tile"],
                    help="form of the bins: each 8 x 8-tile window's list or every tile's list (auto: autotuned "
                         "with the tile, or window lists at a fixed tile)")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--configs", default="1,2,3,4",
                    help="comma-separated other workloads (1-4) timed after the main one ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-ssim", action="store_true", help="skip the measurement of eq. (2) with its SSIM term")
    ap.add_argument("--no-density", action="store_true",
                    help="skip the measurement of adaptive density control (statistics and densify-and-prune)")
    ap.add_argument("--no-pointcloud", action="store_true",
                    help="skip the measurement of point-cloud densification and Gaussian initialisation")
    ap.add_argument("--no-pyramid", action="store_true",
                    help="skip the measurement of the image pyramid and of the coarse-level iterations")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many eager batched steps (for rocprofv3) and exit")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="with --profile-steps: also copy a buffer of this many bytes (a plain copy kernel of "
                         "known size, to calibrate hardware byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              f"(several GPUs would each take a share of the keyframes and all-reduce the parameter "
              f"gradients before the Adam step)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2409_13055_amd import synthetic as S
    from paper_2409_13055_amd import rasterizer as R
    from paper_2409_13055_amd import autotune as A

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    sc = S.make_config(args.workload)
    log(f"[bench] workload {sc.name}: N={sc.n} views={sc.n_views} px={sc.total_pixels} "
        f"({time.time() - t0:.1f}s to generate)")
    params_gen = R.GaussianParams.from_scene(sc, dev)
    target = R.pack_images(sc.targets, dev)
    params, layout = lay_out(params_gen, args.layout, args.steps)
    # Every timed phase starts from these parameters and a fresh optimiser state: the iterations
    # train the Gaussians, which changes the work per iteration as it goes.
    initial = [t.detach().cpu() for t in params.tensors()]
    with_adam = "adam" in sc.work
    lrs = sc.lrs or dict(S.DEFAULT_LRS)
    tile = args.tile
    lds_batch = args.lds_batch
    tune = None
    if tile == 0:
        tune = A.autotune_tile(params, sc.cameras, target, checkpoint=sc.checkpoint,
                               batches=(1, 2) if lds_batch == 0 else (lds_batch,), lists=args.lists)
        tile, lds_batch, lists = tune["best"], tune["lds_batch"], tune["lists"]
        log(f"[bench] autotune: {tune}")
    elif lds_batch == 0:
        lds_batch = 1
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    if tune is None:
        lists = "window" if args.lists == "auto" else args.lists
    step = R.MappingStep(params, sc.cameras, target, lrs=lrs, tile_size=tile, checkpoint=sc.checkpoint,
                         with_adam=with_adam, lds_batch=lds_batch, lists=lists)
    step.size()
    torch.cuda.synchronize()
    log(f"[bench] pairs M={int(step.frame.d_num_pairs.item())} list entries {step.frame.list_entries()} "
        f"capacity={step.rast.capacity} tile {tile} lds_batch {lds_batch} lists {lists}")

    if args.profile_steps > 0:
        for _ in range(args.profile_steps):
            step.run()
        torch.cuda.synchronize()
        if args.copy_probe > 0:
            src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            log(f"[bench] copy probe: {args.copy_probe} bytes")
        log("[bench] profile steps done")
        return

    def reset(st, p=None, init=None):
        for t, t0 in zip((params if p is None else p).tensors(), initial if init is None else init):
            t.copy_(t0)
        for t in st.grads.tensors():
            t.zero_()
        if st.adam is not None:
            for t in st.adam.exp_avg.tensors() + st.adam.exp_avg_sq.tensors():
                t.zero_()
            st.adam.d_step.zero_()
        torch.cuda.synchronize()

    use_graph = not args.no_graph
    if use_graph:
        step.capture()
    run = step.replay if use_graph else step.run
    reset(step)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    peak_hbm = int(torch.cuda.max_memory_allocated())  # everything the batched iteration holds
    if step.overflowed():
        raise RuntimeError("pair capacity overflowed during the timed steps")
    mpix = sc.total_pixels * 1e-6
    value = mpix / (ms * 1e-3)
    loss = step.loss.sum().item()
    log(f"[bench] batched: {ms:.3f} ms/step, {value:.1f} Mpix*iter/s, loss {loss:.5f}")

    if args.layout == "morton":
        # the same iteration on the set in the order it was generated in
        init_g = [t.detach().cpu() for t in params_gen.tensors()]
        st_g = R.MappingStep(params_gen, sc.cameras, target, lrs=lrs, tile_size=tile, checkpoint=sc.checkpoint,
                             with_adam=with_adam, lds_batch=lds_batch, lists=lists)
        st_g.size()
        if use_graph:
            st_g.capture()
        reset(st_g, params_gen, init_g)
        ms_g = time_graph(st_g.replay if use_graph else st_g.run, args.steps, args.warmup)
        # the stages from the same state as the main breakdown (the iterations train the Gaussians)
        reset(st_g, params_gen, init_g)
        for _ in range(args.warmup):
            st_g.run()
        g_stages, _ = stage_breakdown(st_g, args.steps)
        layout["generated_order"] = {"ms_per_step": round(ms_g, 4), "value": round(mpix / (ms_g * 1e-3), 2),
                                     "speedup_of_morton": round(ms_g / ms, 4), "stages_ms": g_stages}
        log(f"[bench] generated order: {ms_g:.3f} ms/step ({ms_g / ms:.3f}x the Morton-ordered step), "
            f"stages {g_stages}")
        del st_g, init_g
    del params_gen

    lists_info = {"form": lists}
    if lists == "window":
        lists_info.update(items=step.frame.list_entries(), windows=step.rast.total_windows)
    other = "tile" if lists == "window" else "window"
    if True:
        # the same iteration with the bins in the other form
        st_t = R.MappingStep(params, sc.cameras, target, lrs=lrs, tile_size=tile, checkpoint=sc.checkpoint,
                             with_adam=with_adam, lds_batch=lds_batch, lists=other)
        st_t.size()
        if use_graph:
            st_t.capture()
        reset(st_t)
        ms_t = time_graph(st_t.replay if use_graph else st_t.run, args.steps, args.warmup)
        reset(st_t)
        for _ in range(args.warmup):
            st_t.run()
        t_stages, _ = stage_breakdown(st_t, args.steps)
        lists_info[f"{other}_lists"] = {"ms_per_step": round(ms_t, 4), "value": round(mpix / (ms_t * 1e-3), 2),
                                        "ratio_to_chosen": round(ms_t / ms, 4), "stages_ms": t_stages}
        log(f"[bench] {other} lists: {ms_t:.3f} ms/step ({ms_t / ms:.3f}x the {lists}-list step), stages {t_stages}")
        del st_t

    # The same iteration issued eagerly (no graph), for comparison.
    eager_ms = None
    if use_graph:
        reset(step)
        for _ in range(args.warmup):
            step.run()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            step.run()
        e1.record()
        torch.cuda.synchronize()
        eager_ms = e0.elapsed_time(e1) / args.steps
        log(f"[bench] eager (no graph): {eager_ms:.3f} ms/step")

    # Per-call breakdown (eager, events around each C call) and the dominant kernel.
    reset(step)
    for _ in range(args.warmup):
        step.run()
    stages, work = stage_breakdown(step, args.steps)
    log(f"[bench] stages (ms): {stages}")

    per_view = None
    if not args.no_per_view:
        pv = R.PerViewMappingStep(params, sc.cameras, sc.targets, lrs=lrs, tile_size=tile,
                                  checkpoint=sc.checkpoint, with_adam=with_adam, lds_batch=lds_batch, lists=lists)
        pv.size()
        reset(pv)
        ms_pv_eager = time_graph(pv.run, args.steps, args.warmup)
        pv.capture()
        reset(pv)
        ms_pv = time_graph(pv.replay, args.steps, args.warmup)
        if pv.overflowed():
            raise RuntimeError("per-view pair capacity overflowed during the timed steps")
        per_view = {"ms_per_step": round(ms_pv, 4), "value": round(mpix / (ms_pv * 1e-3), 2),
                    "batched_speedup": round(ms_pv / ms, 3), "eager_ms_per_step": round(ms_pv_eager, 4),
                    "batched_speedup_vs_eager": round(ms_pv_eager / ms, 3)}
        log(f"[bench] per-view: graph {ms_pv:.3f} ms/step ({per_view['batched_speedup']}x slower than batched), "
            f"eager {ms_pv_eager:.3f} ms/step")
        del pv

    ssim = None
    if not args.no_ssim:
        # eq. (2) with its SSIM term (lambda 0.2, the 3DGS setup): the same iteration with
        # gs_photometric_loss after the forward (not part of `value`: the workload's loss is L1),
        # and the loss call on its own
        lam = 0.2
        st = R.MappingStep(params, sc.cameras, target, lrs=lrs, tile_size=tile, checkpoint=sc.checkpoint,
                           with_adam=with_adam, ssim_lambda=lam, lds_batch=lds_batch, lists=lists)
        st.size()
        if use_graph:
            st.capture()
        run_s = st.replay if use_graph else st.run
        reset(st)
        for _ in range(args.warmup):
            run_s()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            run_s()
        e1.record()
        torch.cuda.synchronize()
        ms_s = e0.elapsed_time(e1) / args.steps
        for _ in range(args.warmup):
            st.photometric(st.frame.rgb, st.target, lam, st.loss, st.dl_dimage)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            st.photometric(st.frame.rgb, st.target, lam, st.loss, st.dl_dimage)
        e1.record()
        torch.cuda.synchronize()
        ms_l = e0.elapsed_time(e1) / args.steps
        alg = 36 * sc.total_pixels  # image and target read, dL/dimage written: 12 bytes per pixel each
        gbs = alg / (ms_l * 1e-3) / 1e9
        # FP32 arithmetic of the separable 11-tap window per pixel and channel (an FMA counts 2; the
        # halo rows the tiles recompute are not counted): forward 5 maps x (11 + 11) FMA + 3 products
        # + ~22 for S and its partials; backward 3 maps x (11 + 11) FMA + ~8 to combine them
        flops = (5 * 22 * 2 + 3 + 22 + 3 * 22 * 2 + 8) * 3 * sc.total_pixels
        tfs = flops / (ms_l * 1e-3) / 1e12
        ssim = {"lambda": lam, "ms_per_step": round(ms_s, 4), "value": round(mpix / (ms_s * 1e-3), 2),
                "loss_call_ms": round(ms_l, 4), "loss_alg_bytes": alg, "loss_GBps": round(gbs, 1),
                "loss_hbm_frac": round(gbs / 8000.0, 4), "loss_flops": flops, "loss_TFLOPs": round(tfs, 2),
                "loss_alu_frac": round(tfs / VALU_PEAK_TFLOPS, 4),
                "loss_alu_frac_without_packed_fp32": round(tfs / VALU_UNPACKED_TFLOPS, 4)}
        log(f"[bench] with SSIM (lambda {lam}): {ms_s:.3f} ms/step; loss call {ms_l:.3f} ms ({gbs:.0f} GB/s alg)")
        del st

    pyramid = None
    if not args.no_pyramid:
        # the Gaussian pyramid of the targets (Sec. III-B): one reduction of every view (the kernel),
        # and the same iteration at the coarse levels the first iterations train on
        pyr = R.ImagePyramid(sc.cameras, target, 2, device=dev)
        for _ in range(args.warmup):
            pyr.reduce_level(0)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            pyr.reduce_level(0)
        e1.record()
        torch.cuda.synchronize()
        ms_r = e0.elapsed_time(e1) / args.steps
        px1 = sum(c.width * c.height for c in pyr.cameras[1])
        alg = 12 * (sc.total_pixels + px1)  # three FP32 channels read at level 0, written at level 1
        gbs = alg / (ms_r * 1e-3) / 1e9
        pyramid = {"reduce_call_ms": round(ms_r, 4), "reduce_alg_bytes": alg, "reduce_GBps": round(gbs, 1),
                   "reduce_hbm_frac": round(gbs / 8000.0, 4), "levels": {}}
        log(f"[bench] pyramid reduce (all views, level 0 -> 1): {ms_r:.4f} ms ({gbs:.0f} GB/s alg)")
        for lv in (1, 2):
            # a coarse level is a different problem (a quarter or a sixteenth of the pixels, the same
            # Gaussians): with the tile size left to the autotuner, each level gets its own choice
            t_lv, b_lv, f_lv, tune_lv = tile, lds_batch, lists, None
            if args.tile == 0:
                tune_lv = A.autotune_tile(params, pyr.cameras[lv], pyr.images[lv], checkpoint=sc.checkpoint,
                                          batches=(1, 2) if args.lds_batch == 0 else (args.lds_batch,),
                                          lists=args.lists, iters=2)
                t_lv, b_lv, f_lv = tune_lv["best"], tune_lv["lds_batch"], tune_lv["lists"]
            st = R.MappingStep(params, pyr.cameras[lv], pyr.images[lv], lrs=lrs, tile_size=t_lv,
                               checkpoint=sc.checkpoint, with_adam=with_adam, lds_batch=b_lv, lists=f_lv)
            st.size()
            if use_graph:
                st.capture()
            run_l = st.replay if use_graph else st.run
            reset(st)
            for _ in range(args.warmup):
                run_l()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                run_l()
            e1.record()
            torch.cuda.synchronize()
            ms_lv = e0.elapsed_time(e1) / args.steps
            pxl = sum(c.width * c.height for c in pyr.cameras[lv])
            pyramid["levels"][str(lv)] = {"ms_per_step": round(ms_lv, 4), "pixels_per_step": pxl,
                                          "value": round(pxl * 1e-6 / (ms_lv * 1e-3), 2),
                                          "speedup_vs_level0": round(ms / ms_lv, 3),
                                          "tile": t_lv, "lds_batch": b_lv, "lists": f_lv}
            if tune_lv is not None:
                pyramid["levels"][str(lv)]["autotune_ms"] = tune_lv["ms_fwd_bwd"]
            log(f"[bench] level {lv}: {ms_lv:.3f} ms/step ({ms / ms_lv:.2f}x faster than level 0; "
                f"tile {t_lv}, batch {b_lv}, {f_lv} lists)")
            del st
        del pyr

    density = None
    if not args.no_density and with_adam:
        # adaptive density control (Sec. III-B): the iteration with its statistics (homodirectional
        # gradient in the raster backward, gs_density_accumulate), then one densify-and-prune step
        # (plan, apply) on the statistics those iterations gathered
        dc = R.DensityControl(params.n, sc.cameras, device=dev)
        st = R.MappingStep(params, sc.cameras, target, lrs=lrs, tile_size=tile, checkpoint=sc.checkpoint,
                           with_adam=with_adam, density=dc, lds_batch=lds_batch, lists=lists)
        st.size()
        if use_graph:
            st.capture()
        run_d = st.replay if use_graph else st.run
        reset(st)
        for t in (dc.grad_accum, dc.abs_accum, dc.count):
            t.zero_()
        for _ in range(args.warmup):
            run_d()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            run_d()
        e1.record()
        torch.cuda.synchronize()
        ms_d = e0.elapsed_time(e1) / args.steps
        st_stages, _ = stage_breakdown(st, args.steps)
        kept, cloned, split = dc.plan(params)
        e0.record()
        for _ in range(args.steps):
            dc.plan_launch(params)
        e1.record()
        torch.cuda.synchronize()
        ms_plan = e0.elapsed_time(e1) / args.steps
        n_out = kept + cloned + 2 * split
        D = params.sh_degree
        outs = [R.GaussianParams.empty(n_out, D, dev) for _ in range(3)]
        eps = torch.randn(split, 2, 3, device=dev)
        dc.plan_launch(params)
        e0.record()
        for _ in range(args.steps):
            dc.apply_into(params, st.adam, eps, *outs)
        e1.record()
        torch.cuda.synchronize()
        ms_apply = e0.elapsed_time(e1) / args.steps
        pn = 11 + 3 * (D + 1) ** 2
        # parameters and both moments: rows read for every surviving source, rows written for the new set
        alg = 3 * 4 * pn * (kept + cloned + split) + 3 * 4 * pn * n_out
        gbs = alg / (ms_apply * 1e-3) / 1e9
        density = {"ms_per_step": round(ms_d, 4), "value": round(mpix / (ms_d * 1e-3), 2),
                   "overhead_vs_value": round(ms_d / ms - 1.0, 4),
                   "raster_bwd_abs_ms": st_stages["raster_bwd"],
                   "project_bwd_adam_stats_ms": st_stages["project_bwd_adam"],
                   "plan_ms": round(ms_plan, 4), "apply_ms": round(ms_apply, 4), "apply_alg_bytes": alg,
                   "apply_GBps": round(gbs, 1), "apply_hbm_frac": round(gbs / 8000.0, 4),
                   "counts": {"kept": kept, "cloned": cloned, "split": split, "n_out": n_out},
                   "statistics_iterations": args.warmup + 2 * args.steps}
        log(f"[bench] density tracking: {ms_d:.3f} ms/step (raster_bwd_abs {st_stages['raster_bwd']} ms, "
            f"project_bwd_adam with statistics {st_stages['project_bwd_adam']} ms); plan {ms_plan:.3f} ms, "
            f"apply {ms_apply:.3f} ms "
            f"({gbs:.0f} GB/s alg), {kept}+{cloned}+2x{split} -> {n_out}")
        del st, outs, dc

    pointcloud = None
    if not args.no_pointcloud:
        # one keyframe's densification (Sec. III-A) and the new Gaussians (Sec. III-B): 3000 tracked
        # pixels of a 1200 x 680 view, every fourth pixel initialised
        cam0 = sc.cameras[0]
        xy, dep, img0 = S.tracked_keyframe(7, cam0.width, cam0.height, 3000)
        pc = R.PointCloudInit(cam0, device=dev)
        image0 = torch.as_tensor(img0.reshape(-1), device=dev)
        t_host = time.perf_counter()
        for _ in range(args.steps):
            pc.triangulate(xy)
        ms_tri = (time.perf_counter() - t_host) * 1e3 / args.steps
        pc.densify(xy, dep, image0, tris=pc.tris)
        n_new = pc.count(4)
        out0 = R.GaussianParams.empty(n_new, sc.sh_degree, dev)
        for _ in range(args.warmup):
            pc.fill(image0)
            pc.init_into(image0, 4, out0)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            pc.fill(image0)
        e1.record()
        torch.cuda.synchronize()
        ms_fill = e0.elapsed_time(e1) / args.steps
        e0.record()
        for _ in range(args.steps):
            pc.init_into(image0, 4, out0)
        e1.record()
        torch.cuda.synchronize()
        ms_init = e0.elapsed_time(e1) / args.steps
        px0 = cam0.width * cam0.height
        pn = 11 + 3 * (sc.sh_degree + 1) ** 2
        pointcloud = {"tracked": int(xy.shape[0]), "triangles": int(pc.tris.shape[0]), "new_gaussians": n_new,
                      "delaunay_host_ms": round(ms_tri, 3), "densify_ms": round(ms_fill, 4),
                      "init_ms": round(ms_init, 4),
                      "densify_alg_bytes": px0 * (12 + 4 + 1), "init_alg_bytes": px0 * (4 + 1) + n_new * (4 * pn + 12)}
        log(f"[bench] point cloud: Delaunay of {xy.shape[0]} points {ms_tri:.2f} ms (host), depth fill "
            f"{ms_fill:.3f} ms, initialisation of {n_new} Gaussians {ms_init:.3f} ms")
        del pc, out0

    roof = roofline(step, sc, stages, work, ms, args.layout)
    others = {}
    for idx in [int(x) for x in args.configs.split(",") if x.strip()]:
        if idx != args.workload:
            others[str(idx)] = bench_config(idx, args)
    cpu = None if args.no_cpu_baseline else cpu_baseline(sc, tile)
    out = {
        "metric": "3DGS fwd+bwd+Adam Mpix*iter/s at 1 GPU (batched HIP-graph step)",
        "value": round(value, 2),
        "unit": "Mpix*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sc.name, "gaussians": sc.n, "views": sc.n_views, "pixels_per_step": sc.total_pixels,
                   "sh_degree": sc.sh_degree, "work": sc.work, "checkpoint": sc.checkpoint, "tile": tile,
                   "lds_batch": lds_batch, "graph": use_graph, "pairs": int(step.frame.d_num_pairs.item()),
                   "layout": args.layout, "lists": lists},
        "layout": layout,
        "lists": lists_info,
        "eager_ms_per_step": None if eager_ms is None else round(eager_ms, 4),
        "peak_hbm_bytes": peak_hbm,
        "per_view": per_view,
        "ssim": ssim,
        "pyramid": pyramid,
        "density": density,
        "pointcloud": pointcloud,
        "stages_ms": stages,
        "roofline": roof,
        "cpu_baseline": cpu,
        "configs": others,
    }
    if tune is not None:
        out["autotune"] = tune
    print(json.dumps(out), flush=True)


def lay_out(params, layout, reps):
    """The Gaussian set in the memory layout `layout` names, and what putting it there costs: for
    "morton" gs_spatial_order and the row gathers of the parameters (the mapping loop also gathers
    both Adam moments, three times the gather bytes), timed over `reps` calls."""
    import torch
    from paper_2409_13055_amd import rasterizer as R
    if layout != "morton":
        return params, {"order": layout}
    out, _, _ = R.spatially_ordered(params)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        order = params.spatial_order()
    e1.record()
    torch.cuda.synchronize()
    ms_order = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        params.gathered(order)
    e1.record()
    torch.cuda.synchronize()
    ms_gather = e0.elapsed_time(e1) / reps
    row = sum(t.numel() for t in params.tensors()) * 4
    log(f"[bench] Morton order of {params.n} Gaussians: order {ms_order:.3f} ms, gather {ms_gather:.3f} ms")
    return out, {"order": layout, "spatial_order_ms": round(ms_order, 4), "gather_params_ms": round(ms_gather, 4),
                 "gather_alg_bytes": 2 * row + 4 * params.n,
                 "gather_GBps": round((2 * row + 4 * params.n) / (ms_gather * 1e-3) / 1e9, 1)}


def time_graph(run, steps, warmup):
    """Average ms of `run` over `steps` calls after `warmup` (HIP events on the current stream)."""
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_config(idx, args):
    """One of the other workloads in its own configuration: the whole iteration its work names
    (forward only; forward and backward; or forward, backward and Adam) replayed as one HIP graph,
    ms/step and Mpix*iter/s; for several views also the same iteration issued view by view (as a
    graph of per-view calls, and eagerly).  Algorithmic bytes per step as in the main workload's
    roofline entry."""
    import torch
    from paper_2409_13055_amd import synthetic as S
    from paper_2409_13055_amd import rasterizer as R
    from paper_2409_13055_amd import autotune as A
    from paper_2409_13055_amd import roofline as RF
    dev = torch.device("cuda:0")
    sc = S.make_config(idx)
    params, _ = lay_out(R.GaussianParams.from_scene(sc, dev), args.layout, 1)
    tune = None
    if sc.work == "fwd":
        tile, lds_batch = 16, 1  # the forward-only workload names 16 x 16 tiles
        # (the autotuner times forward and backward; this workload's forward alone, 1 k Gaussians whose
        # tiles walk their whole lists, is faster with tile lists)
        lists = "tile" if args.lists == "auto" else args.lists
        target = None
    else:
        target = R.pack_images(sc.targets, dev)
        tune = A.autotune_tile(params, sc.cameras, target, checkpoint=sc.checkpoint, lists=args.lists)
        tile, lds_batch, lists = tune["best"], tune["lds_batch"], tune["lists"]
    lrs = sc.lrs or dict(S.DEFAULT_LRS)
    mpix = sc.total_pixels * 1e-6
    if sc.work == "fwd":
        rast = R.Rasterizer(sc.cameras, params.n, params.sh_degree, tile_size=tile, checkpoint=sc.checkpoint,
                            device=dev, lds_batch=lds_batch, lists=lists)
        fr = rast.forward(params)

        def run_eager():
            rast.project(params, fr)
            rast.bin_sort(fr)
            rast.render_fwd(fr)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            run_eager()
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            run_eager()
        ms = time_graph(graph.replay, args.steps, args.warmup)
        overflow = int(fr.d_overflow.item()) != 0
        holder = type("H", (), {})()
        holder.frame, holder.rast, holder.params = fr, rast, params
        c = RF.counts(holder, sc)
        stages = ("project", "bin_sort", "render_fwd")
    else:
        step = R.MappingStep(params, sc.cameras, target, lrs=lrs, tile_size=tile, checkpoint=sc.checkpoint,
                             with_adam="adam" in sc.work, lds_batch=lds_batch, lists=lists)
        step.size()
        step.capture()
        ms = time_graph(step.replay, args.steps, args.warmup)
        overflow = step.overflowed()
        c = RF.counts(step, sc)
        stages = ("project", "bin_sort", "render_fwd", "raster_bwd") + \
            (("project_bwd_adam",) if step.fuse_adam else ("project_bwd",))
    if overflow:
        raise RuntimeError(f"workload {idx}: pair capacity overflowed during the timed steps")
    b = RF.algorithmic_bytes(c)
    alg = sum(b[k] for k in stages)
    gbs = alg / (ms * 1e-3) / 1e9
    out = {"workload": sc.name, "work": sc.work, "gaussians": sc.n, "views": sc.n_views,
           "pixels_per_step": sc.total_pixels, "tile": tile, "lds_batch": lds_batch, "layout": args.layout,
           "lists": lists,
           "pairs": c["M"],
           "ms_per_step": round(ms, 4),
           "value": round(mpix / (ms * 1e-3), 2), "unit": "Mpix*iter/s", "step_alg_bytes": alg,
           "step_GBps": round(gbs, 1), "step_hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    if tune is not None:
        out["autotune"] = tune
    log(f"[bench] workload {sc.name}: {ms:.4f} ms/step, {out['value']} Mpix*iter/s (tile {tile})")
    if not args.no_cpu_baseline:
        # the oracle on the whole workload (every view), one run with every core of the process
        import oracle.oracle as O
        P = O.Params.from_scene(sc)
        opts = O.Options(tile=tile)
        t0 = time.perf_counter()
        if sc.work == "fwd":
            O.forward(P, sc.cameras, opts)
        else:
            fb = O.forward_backward_l1(P, sc.cameras, sc.targets, opts)
            if "adam" in sc.work:
                for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
                    z = np.zeros_like(getattr(P, name))
                    O.adam_step(getattr(P, name), fb["grads"][name], z, z, 1, 1e-3)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": round(mpix / dt, 4), "unit": "Mpix*iter/s", "seconds": round(dt, 4),
                             "cores": O.set_threads(0), "kind": "oracle", "sample": "the whole workload, one run"}
        log(f"[bench]   oracle: {dt:.2f} s ({out['cpu_oracle']['value']} Mpix*iter/s)")
    if sc.n_views > 1 and sc.work != "fwd" and not args.no_per_view:
        pv = R.PerViewMappingStep(params, sc.cameras, sc.targets, lrs=lrs, tile_size=tile,
                                  checkpoint=sc.checkpoint, with_adam="adam" in sc.work, lds_batch=lds_batch,
                                  lists=lists)
        pv.size()
        ms_eager = time_graph(pv.run, args.steps, args.warmup)
        pv.capture()
        ms_pv = time_graph(pv.replay, args.steps, args.warmup)
        if pv.overflowed():
            raise RuntimeError(f"workload {idx}: per-view pair capacity overflowed")
        out["per_view"] = {"ms_per_step": round(ms_pv, 4), "value": round(mpix / (ms_pv * 1e-3), 2),
                           "batched_speedup": round(ms_pv / ms, 3), "eager_ms_per_step": round(ms_eager, 4),
                           "batched_speedup_vs_eager": round(ms_eager / ms, 3)}
        log(f"[bench]   per-view: graph {ms_pv:.4f} ms/step, eager {ms_eager:.4f} ms/step")
        del pv
    return out


def stage_breakdown(step, iters):
    """Average duration of each stage of the batched iteration, measured inside
    `iters` eager iterations (HIP events recorded between the stages on the
    stream the kernels are launched on).  Every stage is one call; project,
    render_fwd, raster_bwd, project_bwd, adam and project_bwd_adam (the
    projection backward fused with the Adam step) each launch one kernel (plus
    the one-thread step increment), so their figures are that kernel's launch
    duration in the iteration."""
    import torch
    if step.fuse_adam:
        names = ["project", "bin_sort", "render_fwd", "clear_grad2d", "raster_bwd", "project_bwd_adam"]
    else:
        names = ["project", "bin_sort", "render_fwd", "clear_grad2d", "raster_bwd", "project_bwd"]
        if step.adam is not None:
            names.append("adam")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(iters)]
    counts = torch.zeros(iters, 3, dtype=torch.int64, device=step.params.means.device)
    torch.cuda.synchronize()
    for it in range(iters):
        marks = iter(evs[it][1:])
        evs[it][0].record()
        step.run(mark=lambda name: next(marks).record())
        # the work counts of this iteration's lists, outside the timed stages
        step.rast.render_stats(step.frame, out=counts[it])
    torch.cuda.synchronize()
    out = {}
    for k, name in enumerate(names):
        out[name] = round(sum(e[k].elapsed_time(e[k + 1]) for e in evs) / iters, 4)
    if not step.fuse_adam:
        out["render_bwd"] = round(out["clear_grad2d"] + out["raster_bwd"] + out["project_bwd"], 4)
    out["step_eager"] = round(sum(e[0].elapsed_time(e[-1]) for e in evs) / iters, 4)
    mean = counts.double().mean(dim=0).tolist()
    work = {"evaluated": mean[0], "blended": mean[1], "contrib_prefix": mean[2], "iterations": iters}
    return out, work


def traffic_of(kernel, tile, checkpoint, workload, layout):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, when it was
    taken on the current kernel source and the same layout of the Gaussian set (None otherwise)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2409_13055_amd", "csrc", rec.get("source", "raster.hip"))
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    key = f"{kernel}/{workload}/tile{tile}/ckpt{int(checkpoint)}/{layout}"
    e = rec.get("entries", {}).get(key)
    if not e or e.get("source_sha") != sha:
        return None
    return e.get("bytes_per_launch")


def roofline(step, sc, stages, work, step_ms, layout):
    """Roofline entry for the dominant single-kernel call (by measured duration) and for the whole
    step; the work counts are the mean over the same iterations the durations are."""
    from paper_2409_13055_amd import roofline as RF
    tr = traffic_of("raster_bwd", step.rast.opts.tile_size, sc.checkpoint, sc.name, layout)
    return RF.report(step, sc, stages, hbm_peak_gbs=HBM_PEAK_GBS, valu_peak_tflops=VALU_PEAK_TFLOPS,
                     valu_unpacked_tflops=VALU_UNPACKED_TFLOPS, traffic=tr, work=work, step_ms=step_ms)


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sc, tile, repeats=3):
    """The FP64 oracle timed on the host cores over a bounded sample of the workload: its first
    keyframe rendered from all Gaussians (projection, binning, blending, L1, backward), plus Adam
    over all parameters when the workload steps the optimiser.  Median of `repeats` runs with every
    core of the process's CPU set, and median of `repeats` runs on one thread."""
    import oracle.oracle as O
    cams, tgts = sc.cameras[:1], sc.targets[:1]
    P = O.Params.from_scene(sc)
    opts = O.Options(tile=tile)
    px = sum(c.width * c.height for c in cams)

    lrs = sc.lrs or {}
    groups = (("means", lrs.get("means")), ("log_scales", lrs.get("log_scales")), ("quats", lrs.get("quats")),
              ("opacity_logits", lrs.get("opacity_logits")), ("sh", lrs.get("sh_dc")))

    def once():
        # the optimiser's first step from zero moments (allocated outside the timed region); its
        # results are dropped, so every run repeats the same iteration
        moments = {name: (np.zeros_like(getattr(P, name)), np.zeros_like(getattr(P, name))) for name, _ in groups} \
            if "adam" in sc.work else {}
        t0 = time.perf_counter()
        fb = O.forward_backward_l1(P, cams, tgts, opts)
        for name, lr in groups:
            if name in moments:
                O.adam_step(getattr(P, name), fb["grads"][name], moments[name][0], moments[name][1], 1, lr)
        return time.perf_counter() - t0

    try:
        all_cores = len(os.sched_getaffinity(0))
    except AttributeError:
        all_cores = os.cpu_count() or 1
    legs = {}
    for cores in (all_cores, 1):
        got = O.set_threads(cores)
        runs = [once() for _ in range(repeats)]
        dt = float(np.median(runs))
        legs[cores] = {"value": round(px * 1e-6 / dt, 4), "cores": got, "seconds": [round(r, 2) for r in runs]}
        log(f"[bench] cpu baseline at {got} threads: runs {legs[cores]['seconds']} s")
    O.set_threads(all_cores)
    a, one = legs[all_cores], legs[1]
    return {"value": a["value"], "unit": "Mpix*iter/s", "cores": a["cores"], "kind": "oracle",
            "sample": f"keyframe 0 of {sc.n_views} ({px} px) rendered from all {sc.n} Gaussians, fwd+L1+bwd"
                      + ("+Adam on all parameters" if "adam" in sc.work else "") + f", FP64, median of {repeats} "
                      f"runs ({a['seconds']} s)",
            "single_thread": {"value": one["value"], "cores": 1, "seconds": one["seconds"]},
            "cpu_model": cpu_model()}


if __name__ == "__main__":
    main()
