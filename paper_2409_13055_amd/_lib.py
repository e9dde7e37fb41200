"""ctypes binding of libgs.so (include/gs.h): argument marshalling only.

Every function here has the name of the C entry point it calls and raises
GsError when that call returns a status other than GS_OK.  Importing this
module fails loudly when the HIP library has not been built: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgs.so")

GS_OK, GS_ERR_INVALID_VALUE, GS_ERR_UNSUPPORTED, GS_ERR_CAPACITY, GS_ERR_HIP = range(5)
GS_LOSS_NONE, GS_LOSS_L1, GS_LOSS_EXTERNAL = 0, 1, 2
GS_MAX_VIEWS = 32
GS_REC_FLOATS = 12
GS_NOALLOC_MAX_TILES = 1 << 20  # tiles of gs_render_fwd_noalloc's static per-tile loss scratch
GS_GRAD2D_FLOATS = 9
GS_MAX_ADAM_GROUPS = 8

P = C.c_void_p


class GsError(RuntimeError):
    def __init__(self, fn, status, detail):
        super().__init__(f"{fn} failed: {status} ({detail})")
        self.status = status


class gs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class gs_params(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32), ("means", P),
                ("log_scales", P), ("quats", P), ("opacity_logits", P), ("sh_dc", P), ("sh_rest", P)]


class gs_options(C.Structure):
    _fields_ = [("tile_size", C.c_int32), ("checkpoint", C.c_int32), ("near_plane", C.c_float),
                ("eps2d", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("radius_sigmas", C.c_float), ("frustum_guard", C.c_float), ("bg", C.c_float * 3),
                ("flags", C.c_uint32), ("lds_batch", C.c_int32)]


class gs_projected(C.Structure):
    _fields_ = [("rec", P), ("tiles_touched", P), ("vis", P), ("vis_count", P)]


class gs_bins(C.Structure):
    _fields_ = [("keys", P), ("ids", P), ("ranges", P), ("capacity", C.c_int64), ("d_num_pairs", P),
                ("d_overflow", P), ("items", P), ("win_ranges", P), ("d_num_items", P)]


class gs_image(C.Structure):
    _fields_ = [("rgb", P), ("t_final", P), ("n_contrib", P)]


class gs_loss(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("target", P), ("dl_dimage", P), ("loss_out", P)]


class gs_grads(C.Structure):
    _fields_ = [("means", P), ("log_scales", P), ("quats", P), ("opacity_logits", P), ("sh_dc", P),
                ("sh_rest", P)]


class gs_density_config(C.Structure):
    _fields_ = [("grad_threshold", C.c_float), ("percent_dense", C.c_float), ("min_opacity", C.c_float),
                ("split_scale_div", C.c_float), ("extent", C.c_float)]


class gs_density_stats(C.Structure):
    _fields_ = [("grad_accum", P), ("abs_accum", P), ("count", P)]


class gs_adam_group(C.Structure):
    _fields_ = [("param", P), ("grad", P), ("exp_avg", P), ("exp_avg_sq", P), ("numel", C.c_int64),
                ("lr", C.c_float), ("reserved", C.c_int32)]


GS_AUTOTUNE_MAX_CANDIDATES = 12  # include/gs.h


class gs_autotune_result(C.Structure):
    _K = GS_AUTOTUNE_MAX_CANDIDATES
    _fields_ = [("tile_size", C.c_int32), ("lds_batch", C.c_int32), ("window_lists", C.c_int32),
                ("from_cache", C.c_int32), ("n_candidates", C.c_int32), ("cand_tile", C.c_int32 * _K),
                ("cand_batch", C.c_int32 * _K), ("cand_window", C.c_int32 * _K), ("ms", C.c_float * _K),
                ("pairs", C.c_int64 * _K)]


EXPORTS = ("gs_status_string", "gs_last_error", "gs_abi_version", "gs_default_options", "gs_total_tiles",
           "gs_total_pixels", "gs_total_windows", "gs_bin_sort_workspace_size", "gs_render_fwd_workspace_size",
           "gs_render_bwd_workspace_size", "gs_project", "gs_bin_sort", "gs_render_fwd", "gs_render_bwd",
           "gs_raster_bwd", "gs_project_bwd", "gs_render_stats", "gs_adam_step", "gs_project_bwd_adam",
           "gs_photometric_loss_workspace_size", "gs_photometric_loss", "gs_pyramid_camera", "gs_pyramid_reduce",
           "gs_raster_bwd_abs", "gs_project_bwd_adam_stats", "gs_default_density_config", "gs_scene_extent", "gs_density_accumulate",
           "gs_density_workspace_size", "gs_density_plan", "gs_density_apply", "gs_delaunay", "gs_densify_depth",
           "gs_init_gaussians_workspace_size", "gs_init_gaussians_count", "gs_init_gaussians",
           "gs_render_fwd_noalloc", "gs_autotune", "gs_spatial_order_workspace_size", "gs_spatial_order",
           "gs_gather_rows")

GS_ABI_VERSION = 4  # include/gs.h
GS_OPT_WINDOW_LISTS = 1  # gs_options.flags
_lib = None


def load(path: str = LIB_PATH):
    """Load libgs.so once; raises when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           f"(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    pc, pp, po = C.POINTER(gs_camera), C.POINTER(gs_params), C.POINTER(gs_options)
    i32, i64, sz = C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "gs_status_string": (C.c_char_p, [C.c_int]),
        "gs_last_error": (C.c_char_p, []),
        "gs_abi_version": (i32, []),
        "gs_default_options": (None, [po]),
        "gs_total_tiles": (C.c_int, [pc, i32, i32, C.POINTER(i64)]),
        "gs_total_pixels": (C.c_int, [pc, i32, C.POINTER(i64)]),
        "gs_total_windows": (C.c_int, [pc, i32, i32, C.POINTER(i64)]),
        "gs_bin_sort_workspace_size": (C.c_int, [i64, pc, i32, po, i64, C.POINTER(sz)]),
        "gs_render_fwd_workspace_size": (C.c_int, [pc, i32, po, C.POINTER(sz)]),
        "gs_render_bwd_workspace_size": (C.c_int, [i64, i32, C.POINTER(sz)]),
        "gs_project": (C.c_int, [pp, pc, i32, po, C.POINTER(gs_projected), P]),
        "gs_bin_sort": (C.c_int, [C.POINTER(gs_projected), i64, pc, i32, po, C.POINTER(gs_bins), P, sz, P]),
        "gs_render_fwd": (C.c_int, [C.POINTER(gs_projected), i64, C.POINTER(gs_bins), pc, i32, po,
                                    C.POINTER(gs_loss), C.POINTER(gs_image), P, sz, P]),
        "gs_autotune": (C.c_int, [pp, pc, i32, po, P, i32, i32, i32, C.POINTER(gs_autotune_result), P]),
        "gs_spatial_order_workspace_size": (C.c_int, [i64, C.POINTER(sz)]),
        "gs_spatial_order": (C.c_int, [P, i64, P, P, sz, P]),
        "gs_gather_rows": (C.c_int, [P, i64, i32, P, P, P]),
        "gs_render_fwd_noalloc": (C.c_int, [C.POINTER(gs_projected), i64, C.POINTER(gs_bins), pc, i32, po,
                                            C.POINTER(gs_loss), C.POINTER(gs_image), P]),
        "gs_render_bwd": (C.c_int, [pp, C.POINTER(gs_projected), C.POINTER(gs_bins), C.POINTER(gs_image), pc, i32,
                                    po, C.POINTER(gs_loss), C.POINTER(gs_grads), P, sz, P]),
        "gs_raster_bwd": (C.c_int, [C.POINTER(gs_projected), i64, C.POINTER(gs_bins), C.POINTER(gs_image), pc, i32,
                                    po, C.POINTER(gs_loss), P, P]),
        "gs_project_bwd": (C.c_int, [pp, C.POINTER(gs_projected), pc, i32, po, P, C.POINTER(gs_grads), P]),
        "gs_render_stats": (C.c_int, [C.POINTER(gs_projected), i64, C.POINTER(gs_bins), pc, i32, po, P, P]),
        "gs_adam_step": (C.c_int, [C.POINTER(gs_adam_group), i32, C.c_double, C.c_double, C.c_double, P, i32, P]),
        "gs_project_bwd_adam": (C.c_int, [pp, C.POINTER(gs_projected), pc, i32, po, P, C.POINTER(gs_adam_group),
                                          C.c_double, C.c_double, C.c_double, P, P]),
        "gs_photometric_loss_workspace_size": (C.c_int, [pc, i32, C.POINTER(sz)]),
        "gs_photometric_loss": (C.c_int, [pc, i32, P, P, C.c_float, P, P, P, sz, P]),
        "gs_pyramid_camera": (C.c_int, [pc, i32, pc]),
        "gs_pyramid_reduce": (C.c_int, [pc, i32, P, P, P]),
        "gs_raster_bwd_abs": (C.c_int, [C.POINTER(gs_projected), i64, C.POINTER(gs_bins), C.POINTER(gs_image), pc,
                                        i32, po, C.POINTER(gs_loss), P, P, P]),
        "gs_project_bwd_adam_stats": (C.c_int, [pp, C.POINTER(gs_projected), pc, i32, po, P,
                                                C.POINTER(gs_adam_group), C.c_double, C.c_double, C.c_double, P, P,
                                                C.POINTER(gs_density_stats), P]),
        "gs_default_density_config": (None, [C.POINTER(gs_density_config)]),
        "gs_delaunay": (C.c_int, [P, i32, P, i32, C.POINTER(i32)]),
        "gs_densify_depth": (C.c_int, [pc, P, P, i32, P, i32, P, C.c_float, P, P, P]),
        "gs_init_gaussians_workspace_size": (C.c_int, [pc, C.POINTER(sz)]),
        "gs_init_gaussians_count": (C.c_int, [pc, P, P, i32, P, P, sz, P]),
        "gs_init_gaussians": (C.c_int, [pc, P, P, P, i32, i32, i64, C.POINTER(gs_grads), P, sz, P]),
        "gs_scene_extent": (C.c_int, [pc, i32, C.POINTER(C.c_float)]),
        "gs_density_accumulate": (C.c_int, [C.POINTER(gs_projected), i64, pc, i32, P, P,
                                            C.POINTER(gs_density_stats), P]),
        "gs_density_workspace_size": (C.c_int, [i64, C.POINTER(sz)]),
        "gs_density_plan": (C.c_int, [pp, C.POINTER(gs_density_stats), C.POINTER(gs_density_config), P, P, sz, P]),
        "gs_density_apply": (C.c_int, [pp, pp, pp, C.POINTER(gs_density_config), P, i64, i64, C.POINTER(gs_grads),
                                       C.POINTER(gs_grads), C.POINTER(gs_grads), P, sz, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if lib.gs_abi_version() != GS_ABI_VERSION:
        raise RuntimeError(f"{path} implements ABI version {lib.gs_abi_version()}, these bindings version "
                           f"{GS_ABI_VERSION}: rebuild the HIP library")
    _lib = lib
    return lib


def _check(fn, status):
    if status != GS_OK:
        lib = load()
        raise GsError(fn, lib.gs_status_string(status).decode(), lib.gs_last_error().decode())


def default_options(**overrides) -> gs_options:
    o = gs_options()
    load().gs_default_options(C.byref(o))
    for k, v in overrides.items():
        if k == "bg":
            for i in range(3):
                o.bg[i] = float(v[i])
        else:
            setattr(o, k, v)
    return o


def make_cameras(cams) -> C.Array:
    """Host array of gs_camera from objects with R, t, fx, fy, cx, cy, width, height."""
    arr = (gs_camera * len(cams))()
    for k, c in enumerate(cams):
        R = [float(x) for x in __import__("numpy").asarray(c.R).reshape(9)]
        t = [float(x) for x in __import__("numpy").asarray(c.t).reshape(3)]
        for i in range(9):
            arr[k].R[i] = R[i]
        for i in range(3):
            arr[k].t[i] = t[i]
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[k].width, arr[k].height = int(c.width), int(c.height)
    return arr


# --------------------------------------------------------------------------- entry points
def gs_total_tiles(cams, n_views, tile_size) -> int:
    out = C.c_int64(0)
    _check("gs_total_tiles", load().gs_total_tiles(cams, n_views, tile_size, C.byref(out)))
    return out.value


def gs_total_windows(cams, n_views, tile_size) -> int:
    out = C.c_int64()
    _check("gs_total_windows", load().gs_total_windows(cams, n_views, tile_size, C.byref(out)))
    return out.value


def gs_total_pixels(cams, n_views) -> int:
    out = C.c_int64(0)
    _check("gs_total_pixels", load().gs_total_pixels(cams, n_views, C.byref(out)))
    return out.value


def gs_bin_sort_workspace_size(n, cams, n_views, opts, pair_capacity) -> int:
    out = C.c_size_t(0)
    _check("gs_bin_sort_workspace_size",
           load().gs_bin_sort_workspace_size(n, cams, n_views, C.byref(opts), pair_capacity, C.byref(out)))
    return out.value


def gs_render_fwd_workspace_size(cams, n_views, opts) -> int:
    out = C.c_size_t(0)
    _check("gs_render_fwd_workspace_size", load().gs_render_fwd_workspace_size(cams, n_views, C.byref(opts),
                                                                              C.byref(out)))
    return out.value


def gs_render_bwd_workspace_size(n, n_views) -> int:
    out = C.c_size_t(0)
    _check("gs_render_bwd_workspace_size", load().gs_render_bwd_workspace_size(n, n_views, C.byref(out)))
    return out.value


def gs_project(params, cams, n_views, opts, out, stream):
    _check("gs_project", load().gs_project(C.byref(params), cams, n_views, C.byref(opts), C.byref(out), stream))


def gs_bin_sort(proj, n, cams, n_views, opts, bins, workspace, workspace_bytes, stream):
    _check("gs_bin_sort", load().gs_bin_sort(C.byref(proj), n, cams, n_views, C.byref(opts), C.byref(bins),
                                             workspace, workspace_bytes, stream))


def gs_render_fwd(proj, n, bins, cams, n_views, opts, loss, out, workspace, workspace_bytes, stream):
    _check("gs_render_fwd", load().gs_render_fwd(C.byref(proj), n, C.byref(bins), cams, n_views, C.byref(opts),
                                                 C.byref(loss) if loss is not None else None, C.byref(out),
                                                 workspace, workspace_bytes, stream))


def gs_spatial_order_workspace_size(n):
    out = C.c_size_t()
    _check("gs_spatial_order_workspace_size", load().gs_spatial_order_workspace_size(n, C.byref(out)))
    return out.value


def gs_spatial_order(means, n, order, workspace, workspace_bytes, stream):
    _check("gs_spatial_order", load().gs_spatial_order(means, n, order, workspace, workspace_bytes, stream))


def gs_gather_rows(src, n, width, order, dst, stream):
    _check("gs_gather_rows", load().gs_gather_rows(src, n, width, order, dst, stream))


def gs_autotune(params, cams, n_views, opts, target, iters, candidate_mask, refresh, stream):
    out = gs_autotune_result()
    _check("gs_autotune", load().gs_autotune(C.byref(params), cams, n_views, C.byref(opts), target, iters,
                                             candidate_mask, refresh, C.byref(out), stream))
    return out


def gs_render_fwd_noalloc(proj, n, bins, cams, n_views, opts, loss, out, stream):
    _check("gs_render_fwd_noalloc", load().gs_render_fwd_noalloc(C.byref(proj), n, C.byref(bins), cams, n_views,
                                                                 C.byref(opts),
                                                                 C.byref(loss) if loss is not None else None,
                                                                 C.byref(out), stream))


def gs_render_bwd(params, proj, bins, img, cams, n_views, opts, loss, grads, workspace, workspace_bytes, stream):
    _check("gs_render_bwd", load().gs_render_bwd(C.byref(params), C.byref(proj), C.byref(bins),
                                                 C.byref(img) if img is not None else None, cams, n_views,
                                                 C.byref(opts), C.byref(loss), C.byref(grads), workspace,
                                                 workspace_bytes, stream))


def gs_raster_bwd(proj, n, bins, img, cams, n_views, opts, loss, grad2d, stream):
    _check("gs_raster_bwd", load().gs_raster_bwd(C.byref(proj), n, C.byref(bins),
                                                 C.byref(img) if img is not None else None, cams, n_views,
                                                 C.byref(opts), C.byref(loss), grad2d, stream))


def gs_project_bwd(params, proj, cams, n_views, opts, grad2d, grads, stream):
    _check("gs_project_bwd", load().gs_project_bwd(C.byref(params), C.byref(proj), cams, n_views, C.byref(opts),
                                                   grad2d, C.byref(grads), stream))


def gs_render_stats(proj, n, bins, cams, n_views, opts, d_counts, stream):
    _check("gs_render_stats", load().gs_render_stats(C.byref(proj), n, C.byref(bins), cams, n_views, C.byref(opts),
                                                     d_counts, stream))


def gs_adam_step(groups, n_groups, beta1, beta2, eps, d_step, zero_grad, stream):
    _check("gs_adam_step", load().gs_adam_step(groups, n_groups, beta1, beta2, eps, d_step, zero_grad, stream))


def gs_project_bwd_adam(params, proj, cams, n_views, opts, grad2d, groups, beta1, beta2, eps, d_step, stream):
    _check("gs_project_bwd_adam", load().gs_project_bwd_adam(C.byref(params), C.byref(proj), cams, n_views,
                                                             C.byref(opts), grad2d, groups, beta1, beta2, eps,
                                                             d_step, stream))


def gs_photometric_loss_workspace_size(cams, n_views) -> int:
    out = C.c_size_t()
    _check("gs_photometric_loss_workspace_size", load().gs_photometric_loss_workspace_size(cams, n_views,
                                                                                           C.byref(out)))
    return out.value


def gs_photometric_loss(cams, n_views, image, target, lam, loss_out, dl_dimage, workspace, workspace_bytes, stream):
    _check("gs_photometric_loss", load().gs_photometric_loss(cams, n_views, image, target, lam, loss_out, dl_dimage,
                                                             workspace, workspace_bytes, stream))


def gs_pyramid_camera(cam: gs_camera, levels: int) -> gs_camera:
    out = gs_camera()
    _check("gs_pyramid_camera", load().gs_pyramid_camera(C.byref(cam), levels, C.byref(out)))
    return out


def gs_pyramid_reduce(cams, n_views, src, dst, stream):
    _check("gs_pyramid_reduce", load().gs_pyramid_reduce(cams, n_views, src, dst, stream))


def gs_raster_bwd_abs(proj, n, bins, img, cams, n_views, opts, loss, grad2d, abs_grad2d, stream):
    _check("gs_raster_bwd_abs", load().gs_raster_bwd_abs(C.byref(proj), n, C.byref(bins),
                                                         C.byref(img) if img is not None else None, cams, n_views,
                                                         C.byref(opts), C.byref(loss), grad2d, abs_grad2d, stream))


def default_density_config(**overrides) -> gs_density_config:
    c = gs_density_config()
    load().gs_default_density_config(C.byref(c))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def gs_scene_extent(cams, n_views) -> float:
    out = C.c_float()
    _check("gs_scene_extent", load().gs_scene_extent(cams, n_views, C.byref(out)))
    return out.value


def gs_density_accumulate(proj, n, cams, n_views, grad2d, abs_grad2d, stats, stream):
    _check("gs_density_accumulate", load().gs_density_accumulate(C.byref(proj), n, cams, n_views, grad2d, abs_grad2d,
                                                                 C.byref(stats), stream))


def gs_density_workspace_size(n) -> int:
    out = C.c_size_t()
    _check("gs_density_workspace_size", load().gs_density_workspace_size(n, C.byref(out)))
    return out.value


def gs_density_plan(params, stats, cfg, d_counts, workspace, workspace_bytes, stream):
    _check("gs_density_plan", load().gs_density_plan(C.byref(params), C.byref(stats), C.byref(cfg), d_counts,
                                                     workspace, workspace_bytes, stream))


def gs_density_apply(params, exp_avg, exp_avg_sq, cfg, eps, n_eps, n_out, out_params, out_exp_avg, out_exp_avg_sq,
                     workspace, workspace_bytes, stream):
    _check("gs_density_apply", load().gs_density_apply(C.byref(params), C.byref(exp_avg), C.byref(exp_avg_sq),
                                                       C.byref(cfg), eps, n_eps, n_out, C.byref(out_params),
                                                       C.byref(out_exp_avg), C.byref(out_exp_avg_sq), workspace,
                                                       workspace_bytes, stream))


def gs_project_bwd_adam_stats(params, proj, cams, n_views, opts, grad2d, groups, beta1, beta2, eps, d_step,
                              abs_grad2d, stats, stream):
    _check("gs_project_bwd_adam_stats", load().gs_project_bwd_adam_stats(
        C.byref(params), C.byref(proj), cams, n_views, C.byref(opts), grad2d, groups, beta1, beta2, eps, d_step,
        abs_grad2d, C.byref(stats), stream))


def gs_delaunay(xy) -> "np.ndarray":
    """Delaunay triangles of integer points xy [n, 2] (host): int32 [n_tris, 3]."""
    import numpy as np
    pts = np.ascontiguousarray(xy, np.int32)
    n = pts.shape[0]
    cap = max(2 * n, 1)
    tris = np.zeros((cap, 3), np.int32)
    nt = C.c_int32()
    _check("gs_delaunay", load().gs_delaunay(pts.ctypes.data_as(C.c_void_p), n, tris.ctypes.data_as(C.c_void_p), cap,
                                             C.byref(nt)))
    return tris[:nt.value].copy()


def gs_densify_depth(cam, xy, depth, n, tris, n_tris, image, tau, depth_map, tracked, stream):
    _check("gs_densify_depth", load().gs_densify_depth(C.byref(cam), xy, depth, n, tris, n_tris, image, tau, depth_map,
                                                       tracked, stream))


def gs_init_gaussians_workspace_size(cam) -> int:
    out = C.c_size_t()
    _check("gs_init_gaussians_workspace_size", load().gs_init_gaussians_workspace_size(C.byref(cam), C.byref(out)))
    return out.value


def gs_init_gaussians_count(cam, depth_map, tracked, stride, d_count, workspace, workspace_bytes, stream):
    _check("gs_init_gaussians_count", load().gs_init_gaussians_count(C.byref(cam), depth_map, tracked, stride, d_count,
                                                                     workspace, workspace_bytes, stream))


def gs_init_gaussians(cam, depth_map, tracked, image, stride, sh_degree, n_out, out, workspace, workspace_bytes,
                      stream):
    _check("gs_init_gaussians", load().gs_init_gaussians(C.byref(cam), depth_map, tracked, image, stride, sh_degree,
                                                         n_out, C.byref(out), workspace, workspace_bytes, stream))
