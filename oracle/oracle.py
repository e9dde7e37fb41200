"""Python face of the FP64 oracle (test infrastructure only).

Wraps liboracle.so (projection, tile binning, per-pixel blending, analytic
backward, local finite differences) and adds the steps that are plain enough
to state in numpy: the photometric loss of eq. (2) (its L1 term, and its SSIM
term with the analytic gradient), the Adam update the paper takes from
the default 3DGS optimisation setup (Sec. IV-A), one level of the
Gaussian pyramid of ground-truth images used for coarse-to-fine training
(Sec. III-B) with the camera that samples it, and the adaptive density
control of Sec. III-B (AbsGS statistics from the backward's per-pixel
gradient magnitudes, split / clone / prune with the 3DGS parameters), and the
point-cloud densification of Sec. III-A (Delaunay triangles of the tracked
pixels through scipy's Qhull, vertex-mean depth in low-gradient regions) with
the initialisation of new Gaussians from it.

Readings of the paper used here (the paper defers the rasteriser to 3DGS,
Sec. III-B): see the header of oracle.cpp; every threshold is a field of
`Options` below, shared with the HIP path by value.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# GS_ORACLE_LIB points the checker at another build of the same source (the sanitizer test's)
_LIB_PATH = os.environ.get("GS_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
_lib = None

SH_C0 = 0.5 / math.sqrt(math.pi)  # the degree-0 real spherical harmonic
REC_FIELDS = ("mx", "my", "depth", "ca", "cb", "cc", "opacity", "r", "g", "b")
GRAD2D_FIELDS = ("mx", "my", "ca", "cb", "cc", "opacity", "r", "g", "b")

# Per-(view, Gaussian) flag bits (same meaning as in oracle.cpp).
F_CLAMP_RGB = 0x7
F_GUARD_X, F_GUARD_Y = 1 << 3, 1 << 4
F_CULL_NEAR, F_CULL_DET, F_CULL_RECT, F_CULL_QUAT, F_CULL_OPACITY = 1 << 8, 1 << 9, 1 << 10, 1 << 11, 1 << 12
F_NEAR_RADIUS, F_NEAR_RECT, F_NEAR_PLANE = 1 << 16, 1 << 17, 1 << 18
# Per-pixel flag bits.
P_NEAR_ALPHA_MIN, P_NEAR_T_MIN, P_NEAR_ALPHA_MAX, P_NEAR_POWER0 = 1, 2, 4, 8


class OrCamera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class OrOptions(C.Structure):
    _fields_ = [("tile", C.c_int32), ("reserved", C.c_int32), ("near_plane", C.c_double), ("eps2d", C.c_double),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double),
                ("radius_sigmas", C.c_double), ("guard", C.c_double), ("bg", C.c_double * 3)]


@dataclasses.dataclass
class Options:
    """Readings of the constants the paper leaves to the 3DGS rasteriser."""
    tile: int = 16
    near_plane: float = 0.2
    eps2d: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    radius_sigmas: float = 3.0
    guard: float = 1.3
    bg: Sequence[float] = (0.0, 0.0, 0.0)

    def as_c(self) -> OrOptions:
        # Thresholds are used at their FP32 values so both sides compare against one number.
        f = lambda x: float(np.float32(x))  # noqa: E731
        o = OrOptions()
        o.tile = int(self.tile)
        o.near_plane, o.eps2d = f(self.near_plane), f(self.eps2d)
        o.alpha_min, o.alpha_max, o.t_min = f(self.alpha_min), f(self.alpha_max), f(self.t_min)
        o.radius_sigmas, o.guard = f(self.radius_sigmas), f(self.guard)
        for i in range(3):
            o.bg[i] = f(self.bg[i])
        return o


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing; build it with oracle/build.py")
        _lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i64, i32 = C.c_int64, C.c_int32
        _lib.or_project.argtypes = [i64, i32, P, P, P, P, P, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P, P, P]
        _lib.or_bin.argtypes = [i32, i64, P, P, P, P, i32, i64, P, P, P, P]
        _lib.or_render.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P, P, P, P]
        _lib.or_render_backward.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, i64, P, P]
        _lib.or_render_tiles.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P, i64, P, P,
                                         P, P]
        _lib.or_render_backward_tiles.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P,
                                                  i64, P, P]
        _lib.or_render_backward_abs.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P, P,
                                                P]
        _lib.or_project_backward.argtypes = [i64, i32, P, P, P, P, P, C.POINTER(OrCamera), i32,
                                             C.POINTER(OrOptions), P, P, P, P, P, P]
        _lib.or_fd_local.argtypes = [i64, i32, P, P, P, P, P, C.POINTER(OrCamera), i32, C.POINTER(OrOptions), P, i64,
                                     P, P, C.c_double, P, P]
        _lib.or_pixel_counts.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P, P]
        _lib.or_bin_sampled.argtypes = [i32, i64, P, P, P, P, i32, P, i64, P, P, i64, P]
        _lib.or_render_flips.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P, i64, i32,
                                         P, P, P, P]
        _lib.or_render_backward_tiles_flips.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P,
                                                        P, P, i64, P, P, i64, P, P, P, P]
        _lib.or_pixel_decisions.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P, P, P,
                                            P, P]
        _lib.or_find_flips.argtypes = [i32, i64, C.POINTER(OrCamera), C.POINTER(OrOptions), P, P, P, P, i64, P, P,
                                       P, P, P, P]
        _lib.or_sh_basis.argtypes = [i32, i64, P, P, P]
        _lib.or_quat_to_rot.argtypes = [P, P]
        _lib.or_set_threads.argtypes = [i32]
        _lib.or_set_threads.restype = i32
        for f in ("or_project", "or_bin", "or_render", "or_render_backward", "or_project_backward", "or_fd_local",
                  "or_render_tiles", "or_render_backward_tiles", "or_render_backward_abs", "or_bin_sampled",
                  "or_render_flips", "or_pixel_decisions", "or_render_backward_tiles_flips", "or_find_flips"):
            getattr(_lib, f).restype = C.c_int
    return _lib


def set_threads(n: int) -> int:
    """Thread count of the oracle's OpenMP loops (n <= 0 leaves it); returns the count in force."""
    return int(lib().or_set_threads(int(n)))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def cameras_c(cams) -> C.Array:
    arr = (OrCamera * len(cams))()
    for k, c in enumerate(cams):
        R = np.asarray(c.R, np.float64).reshape(9)
        t = np.asarray(c.t, np.float64).reshape(3)
        for i in range(9):
            arr[k].R[i] = float(np.float32(R[i]))
        for i in range(3):
            arr[k].t[i] = float(np.float32(t[i]))
        arr[k].fx, arr[k].fy = float(np.float32(c.fx)), float(np.float32(c.fy))
        arr[k].cx, arr[k].cy = float(np.float32(c.cx)), float(np.float32(c.cy))
        arr[k].width, arr[k].height = int(c.width), int(c.height)
    return arr


def tile_grid(cam, tile):
    return (cam.width + tile - 1) // tile, (cam.height + tile - 1) // tile


def total_tiles(cams, tile):
    return sum(np.prod(tile_grid(c, tile)) for c in cams)


# ---------------------------------------------------------------------------
# Parameters as FP64 arrays.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Params:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray  # [N,K,3]
    sh_degree: int

    @property
    def n(self):
        return self.means.shape[0]

    @staticmethod
    def from_scene(scene) -> "Params":
        return Params(_d(scene.means), _d(scene.log_scales), _d(scene.quats), _d(scene.opacity_logits),
                      _d(scene.sh_full()), int(scene.sh_degree))

    def copy(self) -> "Params":
        return Params(self.means.copy(), self.log_scales.copy(), self.quats.copy(), self.opacity_logits.copy(),
                      self.sh.copy(), self.sh_degree)


def project(params: Params, cam, opts: Options):
    """FP64 projection into one view (see or_project)."""
    n = params.n
    rec = np.zeros((n, 10))
    radius = np.zeros(n, np.int32)
    ext = np.zeros((n, 2), np.int32)
    rect = np.zeros((n, 4), np.int32)
    flags = np.zeros(n, np.uint32)
    cov = np.zeros((n, 3))
    cc = cameras_c([cam])
    oc = opts.as_c()
    rc = lib().or_project(n, params.sh_degree, _p(params.means), _p(params.log_scales), _p(params.quats),
                          _p(params.opacity_logits), _p(params.sh), cc, C.byref(oc), _p(rec), _p(radius), _p(ext), _p(rect),
                          _p(flags), _p(cov))
    assert rc == 0
    return dict(rec=rec, radius=radius, ext=ext, rect=rect, flags=flags, cov=cov)


def project_views(params: Params, cams, opts: Options):
    outs = [project(params, c, opts) for c in cams]
    return {k: np.concatenate([o[k] for o in outs]) for k in outs[0]}


def bin_sort(mean2d_f32, ext, depth_f32, cams, tile, with_keys=True):
    """Tile binning + stable key sort on FP32 records (see or_bin).  ext: [V*N, 2] rect
    half-extents (rx, ry), rx = 0 for culled pairs."""
    n_views = len(cams)
    ext = np.ascontiguousarray(ext, np.int32).reshape(-1, 2)
    vn = ext.shape[0]
    n = vn // n_views
    mean2d = np.ascontiguousarray(mean2d_f32, np.float32).reshape(vn, 2)
    depth = np.ascontiguousarray(depth_f32, np.float32).reshape(vn)
    wh = np.array([[c.width, c.height] for c in cams], np.int32)
    T = int(total_tiles(cams, tile))
    npairs = C.c_int64(0)
    # First call sizes the output.
    dummy = np.zeros(1, np.uint32)
    rng = np.zeros(2 * T, np.uint32)
    lib().or_bin(n_views, n, _p(mean2d), _p(ext), _p(depth), _p(wh), tile, 0, None, _p(dummy), _p(rng),
                 C.byref(npairs))
    M = npairs.value
    keys = np.zeros(max(M, 1), np.uint64)
    ids = np.zeros(max(M, 1), np.uint32)
    ranges = np.zeros(2 * T, np.uint32)
    rc = lib().or_bin(n_views, n, _p(mean2d), _p(ext), _p(depth), _p(wh), tile, M,
                      _p(keys) if with_keys else None, _p(ids), _p(ranges), C.byref(npairs))
    assert rc == 0
    return keys[:M], ids[:M], ranges.reshape(T, 2)


def bin_sampled(mean2d_f32, ext, depth_f32, cams, tile, tiles):
    """Brute-force binning of a sample of tiles (see or_bin_sampled): returns the incidence count
    of every tile [T] and, per listed tile (ascending global ids), its ids in the stable
    (depth bits, id) order."""
    n_views = len(cams)
    ext = np.ascontiguousarray(ext, np.int32).reshape(-1, 2)
    vn = ext.shape[0]
    n = vn // n_views
    mean2d = np.ascontiguousarray(mean2d_f32, np.float32).reshape(vn, 2)
    depth = np.ascontiguousarray(depth_f32, np.float32).reshape(vn)
    wh = np.array([[c.width, c.height] for c in cams], np.int32)
    T = int(total_tiles(cams, tile))
    tiles = np.ascontiguousarray(tiles, np.int64)
    assert np.all(np.diff(tiles) > 0) and tiles[0] >= 0 and tiles[-1] < T
    counts = np.zeros(T, np.int64)
    lens = np.zeros(tiles.shape[0], np.int64)
    cap = 1 << 20
    while True:
        out = np.zeros(cap, np.uint32)
        rc = lib().or_bin_sampled(n_views, n, _p(mean2d), _p(ext), _p(depth), _p(wh), tile, _p(tiles),
                                  tiles.shape[0], _p(counts), _p(out), cap, _p(lens))
        if rc == 0:
            break
        assert rc == 2
        cap *= 4
    offs = np.concatenate([[0], np.cumsum(lens)])
    return counts, [out[offs[k]:offs[k + 1]] for k in range(tiles.shape[0])]


def ranges_from_counts(counts):
    """Tile ranges [first, last + 1) of tiles laid out in order with these incidence counts, (0, 0)
    for an empty tile (the layout of the sorted incidence array)."""
    counts = np.asarray(counts, np.int64)
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    r = np.stack([start, start + counts], axis=1)
    r[counts == 0] = 0
    return r


def render_flips(cams, opts: Options, rec, ids, ranges, pixels, max_alt=8, with_positions=False):
    """One-flip alternatives of the listed pixels (see or_render_flips): n_alt [P] (-1: too many
    near-threshold decisions), alt [P, max_alt, 3] colours, kinds [P, max_alt] P_NEAR_* bits (and
    with_positions: ks [P, max_alt], the list position of each)."""
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    px = np.ascontiguousarray(pixels, np.int64)
    n_alt = np.zeros(px.shape[0], np.int32)
    alt = np.full((px.shape[0], max_alt, 3), np.nan)
    kinds = np.zeros((px.shape[0], max_alt), np.uint32)
    ks = np.full((px.shape[0], max_alt), -1, np.int32)
    oc = opts.as_c()
    rc = lib().or_render_flips(n_views, n, cameras_c(cams), C.byref(oc), _p(rec),
                               _p(np.ascontiguousarray(ids, np.uint32)), _p(np.ascontiguousarray(ranges, np.uint32)),
                               _p(px), px.shape[0], max_alt, _p(n_alt), _p(alt), _p(kinds), _p(ks))
    assert rc == 0
    return (n_alt, alt, kinds, ks) if with_positions else (n_alt, alt, kinds)


def find_flips(cams, opts: Options, rec, ids, ranges, pixels, target_nc, target_T, target_rgb):
    """Per listed pixel, the single decision taken the other way that gives it the contributor count
    target_nc and the final transmittance target_T (see or_find_flips): (found [P] 0/1/-1, positions
    [P], kinds [P])."""
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    px = np.ascontiguousarray(pixels, np.int64)
    tnc = np.ascontiguousarray(target_nc, np.int32)
    tT = np.ascontiguousarray(target_T, np.float64)
    trgb = np.ascontiguousarray(np.asarray(target_rgb, np.float64).reshape(-1, 3))
    found = np.zeros(px.shape[0], np.int32)
    ks = np.zeros(px.shape[0], np.int32)
    kinds = np.zeros(px.shape[0], np.uint32)
    oc = opts.as_c()
    rc = lib().or_find_flips(n_views, n, cameras_c(cams), C.byref(oc), _p(rec),
                             _p(np.ascontiguousarray(ids, np.uint32)), _p(np.ascontiguousarray(ranges, np.uint32)),
                             _p(px), px.shape[0], _p(tnc), _p(tT), _p(trgb), _p(found), _p(ks), _p(kinds))
    assert rc == 0
    return found, ks, kinds


def pixel_decisions(cams, opts: Options, rec, ids, ranges):
    """Per pixel: blended count, order-independent hash of the blended ids, the id that ended the
    pixel (0xffffffff: none), and the smallest relative distances of an alpha from alpha_min and of
    a transmittance from t_min (see or_pixel_decisions)."""
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    P = sum(c.width * c.height for c in cams)
    nb = np.zeros(P, np.int32)
    h = np.zeros(P, np.uint64)
    stop = np.zeros(P, np.uint32)
    ma = np.zeros(P)
    mt = np.zeros(P)
    oc = opts.as_c()
    rc = lib().or_pixel_decisions(n_views, n, cameras_c(cams), C.byref(oc), _p(rec),
                                  _p(np.ascontiguousarray(ids, np.uint32)),
                                  _p(np.ascontiguousarray(ranges, np.uint32)), _p(nb), _p(h), _p(stop), _p(ma), _p(mt))
    assert rc == 0
    return dict(n_blended=nb, blend_hash=h, stop_id=stop, margin_alpha=ma, margin_t=mt)


def render(cams, opts: Options, rec, ids, ranges):
    """Per-pixel front-to-back blending (see or_render).  rec: [V*N,10] FP64."""
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    P = sum(c.width * c.height for c in cams)
    image = np.zeros(3 * P)
    tf = np.zeros(P)
    nc = np.zeros(P, np.int32)
    pf = np.zeros(P, np.uint32)
    ids = np.ascontiguousarray(ids, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    oc = opts.as_c()
    rc = lib().or_render(n_views, n, cameras_c(cams), C.byref(oc), _p(rec), _p(ids), _p(ranges), _p(image), _p(tf),
                         _p(nc), _p(pf))
    assert rc == 0
    return dict(image=image, t_final=tf, n_contrib=nc, pix_flags=pf)


def render_tiles(cams, opts: Options, rec, ids, ranges, tiles):
    """or_render restricted to the global tiles listed; other pixels are NaN."""
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    P = sum(c.width * c.height for c in cams)
    image = np.full(3 * P, np.nan)
    tf = np.full(P, np.nan)
    nc = np.full(P, -1, np.int32)
    pf = np.zeros(P, np.uint32)
    t = np.ascontiguousarray(tiles, np.int64)
    ids = np.ascontiguousarray(ids, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    oc = opts.as_c()
    rc = lib().or_render_tiles(n_views, n, cameras_c(cams), C.byref(oc), _p(rec), _p(ids), _p(ranges), _p(t),
                               t.shape[0], _p(image), _p(tf), _p(nc), _p(pf))
    assert rc == 0
    return dict(image=image, t_final=tf, n_contrib=nc, pix_flags=pf)


def render_backward_tiles(cams, opts: Options, rec, ids, ranges, tiles, dl_dimage, flips=None, with_mag=False):
    """Image-space gradients summed over the pixels of the listed tiles only.  flips: optional
    (pixels, positions, kinds) arrays, one decision per listed pixel taken the other way (see
    or_render_backward_tiles_flips).  with_mag: also return, per row and component, the sum of the
    magnitudes of the per-pixel terms (the scale of the rounding error of any summation of them)."""
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    g2 = np.zeros((n_views * n, 9))
    mag = np.zeros((n_views * n, 9))
    t = np.ascontiguousarray(tiles, np.int64)
    oc = opts.as_c()
    ids = np.ascontiguousarray(ids, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    if flips is None:
        flips = (np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint32))
    order = np.argsort(np.asarray(flips[0], np.int64), kind="stable")
    fp = np.ascontiguousarray(np.asarray(flips[0], np.int64)[order])
    fk = np.ascontiguousarray(np.asarray(flips[1], np.int32)[order])
    fkind = np.ascontiguousarray(np.asarray(flips[2], np.uint32)[order])
    rc = lib().or_render_backward_tiles_flips(n_views, n, cameras_c(cams), C.byref(oc), _p(rec), _p(ids),
                                              _p(ranges), _p(t), t.shape[0], _p(_d(dl_dimage)), _p(g2),
                                              fp.shape[0], _p(fp), _p(fk), _p(fkind), _p(mag))
    assert rc == 0
    return (g2, mag) if with_mag else g2


def render_backward_mag(cams, opts: Options, rec, ids, ranges, dl_dimage):
    """render_backward over every tile with the per-row, per-component sums of the magnitudes of the
    per-pixel terms (see render_backward_tiles)."""
    T = int(total_tiles(cams, opts.tile))
    return render_backward_tiles(cams, opts, rec, ids, ranges, np.arange(T), dl_dimage, with_mag=True)


def pixel_counts(cams, opts: Options, rec, ids, ranges):
    """Per pixel: list entries evaluated until the pixel stops, and entries blended."""
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    P = sum(c.width * c.height for c in cams)
    ev = np.zeros(P, np.int64)
    bl = np.zeros(P, np.int64)
    oc = opts.as_c()
    lib().or_pixel_counts(n_views, n, cameras_c(cams), C.byref(oc), _p(rec),
                          _p(np.ascontiguousarray(ids, np.uint32)), _p(np.ascontiguousarray(ranges, np.uint32)),
                          _p(ev), _p(bl))
    return ev, bl


def split_views(flat, cams, channels=3):
    """Split a packed per-view buffer into a list of [channels,H,W] (or [H,W]) arrays."""
    out, off = [], 0
    for c in cams:
        k = channels * c.width * c.height
        a = flat[off:off + k]
        out.append(a.reshape(channels, c.height, c.width) if channels > 1 else a.reshape(c.height, c.width))
        off += k
    return out


def pack_views(arrs) -> np.ndarray:
    return np.concatenate([np.asarray(a, np.float64).reshape(-1) for a in arrs])


def l1_loss(image_flat, targets, cams):
    """L1 term of eq. (2): sum over views of the per-view mean |I_r - I_gt|.

    Returns (loss, dL/dimage) with the gradient sign(I_r - I_gt)/(3 H W), sign(0) = 0.
    """
    tgt = pack_views(targets)
    d = image_flat - tgt
    w = np.concatenate([np.full(3 * c.width * c.height, 1.0 / (3.0 * c.width * c.height)) for c in cams])
    return float(np.sum(w * np.abs(d))), w * np.sign(d)


def l1_loss_per_view(image_flat, targets, cams):
    tgt = pack_views(targets)
    out, off = [], 0
    for c in cams:
        k = 3 * c.width * c.height
        out.append(float(np.sum(np.abs(image_flat[off:off + k] - tgt[off:off + k])) / k))
        off += k
    return out


# ---------------------------------------------------------------------------
# The SSIM term of eq. (2).  The paper prints the loss garbled; the reading is
# (1 - lambda) L1 + lambda (1 - SSIM) with lambda = 0.2 (the 3DGS setup it adopts,
# Sec. IV-A), SSIM computed as in the 3DGS loss: per channel, an 11 x 11 Gaussian
# window (sigma 1.5, normalised), zero-padded same-size filtering, C1 = 0.01^2,
# C2 = 0.03^2, the map averaged over the view's pixels and channels.
# ---------------------------------------------------------------------------
SSIM_TAPS = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window():
    """1D Gaussian window: 11 taps, sigma 1.5, normalised to sum 1 (the 2D window is its outer product)."""
    t = np.arange(SSIM_TAPS, dtype=np.float64) - SSIM_TAPS // 2
    g = np.exp(-t * t / (2.0 * SSIM_SIGMA * SSIM_SIGMA))
    return g / g.sum()


def ssim_blur(img):
    """Window-weighted sum around every pixel of img [H, W] (zero outside the image), same size."""
    g = ssim_window()
    r = SSIM_TAPS // 2
    H, W = img.shape
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    rows = sum(g[t] * pad[:, t:t + W] for t in range(SSIM_TAPS))  # along x: [H + 2r, W]
    return sum(g[t] * rows[t:t + H, :] for t in range(SSIM_TAPS))  # along y: [H, W]


def ssim_map(x, y):
    """SSIM at every pixel of one channel; also returns its partial derivatives with respect to the
    local statistics of x: A = dS/dmu_x, B = dS/dE[x^2], C = dS/dE[xy] (the y statistics held)."""
    mx, my = ssim_blur(x), ssim_blur(y)
    exx, eyy, exy = ssim_blur(x * x), ssim_blur(y * y), ssim_blur(x * y)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    n1, n2 = 2.0 * mx * my + SSIM_C1, 2.0 * sxy + SSIM_C2
    d1, d2 = mx * mx + my * my + SSIM_C1, sxx + syy + SSIM_C2
    s = n1 * n2 / (d1 * d2)
    # chain rule through sxx = E[x^2] - mu_x^2 and sxy = E[xy] - mu_x mu_y
    a = 2.0 * (my * (n2 - n1) - s * mx * (d2 - d1)) / (d1 * d2)
    b = -s / d2
    c = 2.0 * n1 / (d1 * d2)
    return s, a, b, c


def ssim_view(img3, tgt3):
    """Mean SSIM of one view ([3, H, W] each) and its gradient with respect to img3."""
    n = img3.size
    total, grad = 0.0, np.zeros_like(img3, dtype=np.float64)
    for ch in range(3):
        x, y = np.asarray(img3[ch], np.float64), np.asarray(tgt3[ch], np.float64)
        s, a, b, c = ssim_map(x, y)
        total += s.sum()
        # mu_x, E[x^2] and E[xy] at pixel p are window sums over x around p: the adjoint of the
        # zero-padded symmetric window is the same window
        grad[ch] = (ssim_blur(a) + 2.0 * x * ssim_blur(b) + y * ssim_blur(c)) / n
    return total / n, grad


def photometric_loss(image_flat, targets, cams, lam):
    """eq. (2) read as (1 - lam) L1 + lam (1 - SSIM) per view, summed over views.

    Returns (per-view losses, dL/dimage) in the packed planar layout of the images."""
    tgt = pack_views(targets)
    img = np.asarray(image_flat, np.float64)
    losses, grad, off = [], np.zeros_like(img), 0
    for cam in cams:
        k = 3 * cam.width * cam.height
        x = img[off:off + k].reshape(3, cam.height, cam.width)
        y = tgt[off:off + k].reshape(3, cam.height, cam.width)
        ssim, gs = ssim_view(x, y)
        d = (x - y).reshape(-1)
        losses.append((1.0 - lam) * float(np.abs(d).sum()) / k + lam * (1.0 - ssim))
        grad[off:off + k] = (1.0 - lam) * np.sign(d) / k - lam * gs.reshape(-1)
        off += k
    return losses, grad


# ---------------------------------------------------------------------------
# Gaussian-pyramid training (Sec. III-B, after Photo-SLAM): the ground-truth image
# repeatedly smoothed and down-sampled, coarse levels used first.  Reading: one
# level is the REDUCE step of Burt and Adelson's Gaussian pyramid, the separable
# binomial window (1, 4, 6, 4, 1)/16 centred on every second pixel, output size
# ceil(W/2) x ceil(H/2), the border reflected without repeating the edge pixel
# (index -1 reads 1, index W reads W - 2).  A level's camera samples output pixel
# x' at input index 2 x', so in index coordinates u' = u / 2: fx' = fx / 2,
# cx' = cx / 2 + 1/4 (a point projects to fx x/z + cx - 1/2), likewise in y.
# ---------------------------------------------------------------------------
PYR_TAPS = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


def _reflect(i, n):
    """Index i reflected into [0, n) without repeating the edge sample."""
    if n == 1:
        return 0
    period = 2 * (n - 1)
    i = abs(i) % period
    return period - i if i >= n else i


def pyramid_reduce(img):
    """One pyramid level of img [C, H, W] (FP64): [C, ceil(H/2), ceil(W/2)]."""
    img = np.asarray(img, np.float64)
    C, H, W = img.shape
    H2, W2 = (H + 1) // 2, (W + 1) // 2
    xs = np.array([[_reflect(2 * x + k - 2, W) for k in range(5)] for x in range(W2)])  # [W2, 5]
    ys = np.array([[_reflect(2 * y + k - 2, H) for k in range(5)] for y in range(H2)])  # [H2, 5]
    rows = np.einsum("k,chxk->chx", PYR_TAPS, img[:, :, xs])                            # [C, H, W2]
    return np.einsum("k,cyxk->cyx", PYR_TAPS, rows[:, ys, :].transpose(0, 1, 3, 2))      # [C, H2, W2]


def pyramid_camera(cam, levels=1):
    """The camera that samples `levels` REDUCE steps of cam's image."""
    for _ in range(levels):
        cam = dataclasses.replace(cam, fx=cam.fx / 2.0, fy=cam.fy / 2.0, cx=cam.cx / 2.0 + 0.25,
                                  cy=cam.cy / 2.0 + 0.25, width=(cam.width + 1) // 2,
                                  height=(cam.height + 1) // 2)
    return cam


def render_backward(cams, opts: Options, rec, ids, ranges, dl_dimage):
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    g2 = np.zeros((n_views * n, 9))
    ids = np.ascontiguousarray(ids, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    dl = _d(dl_dimage)
    oc = opts.as_c()
    rc = lib().or_render_backward(n_views, n, cameras_c(cams), C.byref(oc), _p(rec), _p(ids), _p(ranges),
                                  int(ids.shape[0]), _p(dl), _p(g2))
    assert rc == 0
    return g2


def render_backward_abs(cams, opts: Options, rec, ids, ranges, dl_dimage):
    """render_backward plus the homodirectional view-space gradient of AbsGS: abs2d [V*N][2], per
    (view, Gaussian) the sums over pixels of |dL_p/dmx| and |dL_p/dmy| (pixel units)."""
    n_views = len(cams)
    rec = _d(rec)
    n = rec.shape[0] // n_views
    g2 = np.zeros((n_views * n, 9))
    a2 = np.zeros((n_views * n, 2))
    oc = opts.as_c()
    rc = lib().or_render_backward_abs(n_views, n, cameras_c(cams), C.byref(oc), _p(rec),
                                      _p(np.ascontiguousarray(ids, np.uint32)),
                                      _p(np.ascontiguousarray(ranges, np.uint32)), _p(_d(dl_dimage)), _p(g2), _p(a2))
    assert rc == 0
    return g2, a2


# ---------------------------------------------------------------------------
# Adaptive density control (Sec. III-B): AbsGS densification with the 3DGS
# split/clone parameters, pruning by opacity.  Readings (the paper names the
# method and says the 3DGS parameters are kept):
#  - statistics as in 3DGS, one observation per (view, Gaussian) pair whose
#    Gaussian touches a tile of the view: the view-space gradient is the mean's
#    gradient in normalised device units, (W/2) dL/dmx and (H/2) dL/dmy; the
#    homodirectional one takes AbsGS's per-pixel magnitudes instead; each adds
#    its Euclidean norm to an accumulator and the pair adds 1 to a count;
#  - a Gaussian is selected when its mean homodirectional norm reaches tau
#    (3DGS: 0.0002), decided in FP32 as accum >= tau * count (count > 0);
#  - selected and max scale > percent_dense * extent (3DGS: 0.01; extent 1.1
#    times the largest distance of a camera centre from their mean): split into
#    two, each with mean mu + R (s * eps) (eps a standard normal draw, passed in)
#    and scales s / 1.6; selected and not larger: cloned (an exact copy); the
#    scale test is taken in FP32 on log scales against log(percent_dense *
#    extent);
#  - opacity below 0.005 (FP32 test on the logit against logit(0.005)): pruned,
#    with no clone or split (children inherit the opacity, so 3DGS prunes them
#    too);
#  - output order: the kept originals, the clones, every split's first child,
#    every split's second child, each in the original order; Adam moments are
#    kept for originals and zero for new Gaussians; the statistics restart at 0.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class DensityConfig:
    extent: float
    grad_threshold: float = 0.0002
    percent_dense: float = 0.01
    min_opacity: float = 0.005
    split_scale_div: float = 1.6


def scene_extent(cams):
    """1.1 times the largest distance of a camera centre from the centres' mean."""
    c = np.array([-np.asarray(cm.R, np.float64).T @ np.asarray(cm.t, np.float64) for cm in cams])
    return 1.1 * float(np.max(np.linalg.norm(c - c.mean(0), axis=1)))


def density_accumulate(grad_acc, abs_acc, count, tiles_touched, grad2d, abs2d, cams):
    """Adds one iteration's view-space gradient norms to the per-Gaussian statistics (in place)."""
    n = grad_acc.shape[0]
    for v, c in enumerate(cams):
        sl = slice(v * n, (v + 1) * n)
        vis = np.asarray(tiles_touched[sl]) > 0
        sx, sy = c.width / 2.0, c.height / 2.0
        g = np.hypot(sx * grad2d[sl, 0], sy * grad2d[sl, 1])
        a = np.hypot(sx * abs2d[sl, 0], sy * abs2d[sl, 1])
        grad_acc[vis] += g[vis]
        abs_acc[vis] += a[vis]
        count[vis] += 1


def density_classes(params: Params, abs_acc, count, cfg: DensityConfig):
    """(keep, clone, split) masks; every decision in FP32 as stated in the readings above."""
    f = np.float32
    sel = (np.asarray(count) > 0) & (np.asarray(abs_acc, f) >= f(cfg.grad_threshold) * np.asarray(count, f))
    large = np.asarray(params.log_scales, f).max(axis=1) > f(math.log(cfg.percent_dense * cfg.extent))
    pruned = np.asarray(params.opacity_logits, f).reshape(-1) < f(math.log(cfg.min_opacity / (1.0 - cfg.min_opacity)))
    keep = ~pruned & ~(sel & large)
    return keep, ~pruned & sel & ~large, ~pruned & sel & large


def densify_and_prune(params: Params, exp_avg: Params, exp_avg_sq: Params, abs_acc, count, cfg: DensityConfig,
                      eps):
    """One density-control step.  eps [n_split, 2, 3]: the standard normal draws of the split
    children, in split order (first child, second child).  Returns the new parameters and moments
    (as Params) and the three masks."""
    keep, clone, split = density_classes(params, abs_acc, count, cfg)
    ns = int(split.sum())
    eps = np.asarray(eps, np.float64).reshape(ns, 2, 3)
    q = params.quats[split]
    R = np.array([quat_to_rot(qq / np.linalg.norm(qq)) for qq in q]).reshape(ns, 3, 3)
    s = np.exp(params.log_scales[split])

    def build(arrs, child):
        return [np.concatenate([a[keep], a[clone]] + [child(a, k) for k in range(2)]) for a in arrs]

    def child_param(name):
        def f(a, k):
            if name == "means":
                return a[split] + np.einsum("nij,nj->ni", R, s * eps[:, k, :])
            if name == "log_scales":
                return a[split] - math.log(cfg.split_scale_div)
            return a[split]
        return f

    names = ("means", "log_scales", "quats", "opacity_logits", "sh")
    out = {k: build([getattr(params, k)], child_param(k))[0] for k in names}
    new_p = Params(out["means"], out["log_scales"], out["quats"], out["opacity_logits"], out["sh"], params.sh_degree)

    def moments(m):
        o = {}
        for k in names:
            a = getattr(m, k)
            o[k] = np.concatenate([a[keep]] + [np.zeros((int(clone.sum()) + 2 * ns,) + a.shape[1:])])
        return Params(o["means"], o["log_scales"], o["quats"], o["opacity_logits"], o["sh"], m.sh_degree)

    return new_p, moments(exp_avg), moments(exp_avg_sq), (keep, clone, split)


# ---------------------------------------------------------------------------
# Point-cloud densification and Gaussian initialisation (Sec. III-A, Sec. III-B).
# The paper triangulates the image with the tracked pixels as vertices
# (Delaunay), gives each pixel of a low-gradient region the mean depth of its
# triangle's vertices, and initialises new Gaussians at the points with their
# colour.  Readings:
#  - tracked pixels have integer pixel coordinates, distinct, not all
#    collinear; the triangulation is the Delaunay triangulation of their
#    convex hull (any one of the valid ones where four are cocircular);
#  - a pixel belongs to the triangle whose closed interior holds it, edges
#    shared by two triangles going to one of them: an edge a -> b of a
#    triangle with positive orientation is its own when b.y > a.y, or b.y ==
#    a.y and b.x < a.x (exact integer tests); a tracked pixel keeps its own
#    depth and is never interpolated;
#  - low gradient: grey = (r + g + b) / 3, central differences (one-sided at
#    the border) gx, gy, and gx^2 + gy^2 < tau^2, every step in FP32;
#  - a new Gaussian per pixel with a depth (tracked or interpolated) on the
#    grid of stride `stride` (x % stride == 0 and y % stride == 0; tracked
#    pixels always), in row-major pixel order: mean = the pixel's index
#    coordinate unprojected at its depth, sh_dc = (colour - 1/2) / SH_C0,
#    identity rotation, opacity 0.1 (the 3DGS initial opacity), isotropic
#    scale of the pixel footprint, stride * depth / fx, higher SH bands 0.
# ---------------------------------------------------------------------------
def delaunay_triangles(pts):
    """Delaunay triangles of integer points [n, 2] (scipy's Qhull), as sorted index triples."""
    from scipy.spatial import Delaunay
    tri = Delaunay(np.asarray(pts, np.float64)).simplices
    return np.unique(np.sort(tri, axis=1), axis=0)


def _orient(a, b, c):
    return (int(b[0]) - int(a[0])) * (int(c[1]) - int(a[1])) - (int(b[1]) - int(a[1])) * (int(c[0]) - int(a[0]))


def pixel_owner(pts, tris, W, H):
    """Per pixel the index of the triangle that owns it, -1 if none (exact integer edge tests)."""
    pts = np.asarray(pts, np.int64)
    owner = np.full((H, W), -1, np.int64)
    for t, (i, j, k) in enumerate(tris):
        a, b, c = pts[i], pts[j], pts[k]
        if _orient(a, b, c) < 0:
            b, c = c, b
        # only pixels of the triangle's bounding box can be inside it
        x0, x1 = max(0, min(a[0], b[0], c[0])), min(W - 1, max(a[0], b[0], c[0]))
        y0, y1 = max(0, min(a[1], b[1], c[1])), min(H - 1, max(a[1], b[1], c[1]))
        if x1 < x0 or y1 < y0:
            continue
        yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        inside = np.ones(yy.shape, bool)
        for u, v in ((a, b), (b, c), (c, a)):
            e = (v[0] - u[0]) * (yy - u[1]) - (v[1] - u[1]) * (xx - u[0])
            own = v[1] > u[1] or (v[1] == u[1] and v[0] < u[0])
            inside &= (e > 0) | ((e == 0) & own)
        box = owner[y0:y1 + 1, x0:x1 + 1]
        assert not np.any(box[inside] >= 0), "a pixel owned twice"
        box[inside] = t
    return owner


def low_gradient_mask(img3, tau):
    """gx^2 + gy^2 < tau^2 of the grey image, every step in FP32 as stated above."""
    f = np.float32
    im = np.asarray(img3, f)
    grey = (im[0] + im[1] + im[2]) / f(3.0)
    H, W = grey.shape
    gx = np.empty_like(grey)
    gy = np.empty_like(grey)
    if W > 1:
        gx[:, 1:-1] = (grey[:, 2:] - grey[:, :-2]) * f(0.5)
        gx[:, 0] = grey[:, 1] - grey[:, 0]
        gx[:, -1] = grey[:, -1] - grey[:, -2]
    else:
        gx[:] = 0
    if H > 1:
        gy[1:-1] = (grey[2:] - grey[:-2]) * f(0.5)
        gy[0] = grey[1] - grey[0]
        gy[-1] = grey[-1] - grey[-2]
    else:
        gy[:] = 0
    return gx * gx + gy * gy < f(tau) * f(tau)


def interpolate_depth(pts, depths, tris, img3, tau):
    """Depth map [H, W] (0 where none): tracked pixels their depth, low-gradient pixels the mean
    depth of the vertices of the triangle that owns them."""
    H, W = img3.shape[1:]
    owner = pixel_owner(pts, tris, W, H)
    mask = low_gradient_mask(img3, tau)
    d = np.asarray(depths, np.float64)
    tri_mean = d[np.asarray(tris)].mean(axis=1) if len(tris) else np.zeros(0)
    out = np.where((owner >= 0) & mask, tri_mean[np.maximum(owner, 0)] if len(tris) else 0.0, 0.0)
    pts = np.asarray(pts, np.int64)
    out[pts[:, 1], pts[:, 0]] = d
    return out, owner


def init_gaussians(depth, img3, cam, stride, tracked_mask):
    """New Gaussians from a depth map (see the readings above): dict of means [m, 3], log_scales
    [m, 3], quats [m, 4], opacity_logits [m], sh_dc [m, 3], and the pixel indices used."""
    H, W = depth.shape
    yy, xx = np.mgrid[0:H, 0:W]
    grid = (xx % stride == 0) & (yy % stride == 0)
    use = (depth > 0) & (grid | tracked_mask)
    idx = np.flatnonzero(use.reshape(-1))
    x, y = xx.reshape(-1)[idx].astype(np.float64), yy.reshape(-1)[idx].astype(np.float64)
    z = depth.reshape(-1)[idx]
    # index coordinate u = fx X/Z + cx - 1/2
    pc = np.stack([(x - cam.cx + 0.5) / cam.fx * z, (y - cam.cy + 0.5) / cam.fy * z, z], 1)
    R, t = np.asarray(cam.R, np.float64), np.asarray(cam.t, np.float64)
    means = (pc - t) @ R
    col = np.asarray(img3, np.float64).reshape(3, -1)[:, idx].T
    m = idx.size
    return dict(means=means, log_scales=np.repeat(np.log(stride * z / cam.fx)[:, None], 3, 1),
                quats=np.tile([1.0, 0.0, 0.0, 0.0], (m, 1)), opacity_logits=np.full(m, math.log(0.1 / 0.9)),
                sh_dc=(col - 0.5) / SH_C0, pixels=idx)


def project_backward(params: Params, cams, opts: Options, grad2d):
    n = params.n
    K = (params.sh_degree + 1) ** 2
    g = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
             opacity_logits=np.zeros(n), sh=np.zeros((n, K, 3)))
    g2 = _d(grad2d)
    oc = opts.as_c()
    rc = lib().or_project_backward(n, params.sh_degree, _p(params.means), _p(params.log_scales), _p(params.quats),
                                   _p(params.opacity_logits), _p(params.sh), cameras_c(cams), len(cams), C.byref(oc),
                                   _p(g2), _p(g["means"]), _p(g["log_scales"]), _p(g["quats"]),
                                   _p(g["opacity_logits"]), _p(g["sh"]))
    assert rc == 0
    return g


def forward(params: Params, cams, opts: Options):
    """Independent FP64 pipeline: project, bin on the FP32-rounded records, blend."""
    pr = project_views(params, cams, opts)
    rec = pr["rec"]
    keys, ids, ranges = bin_sort(rec[:, 0:2].astype(np.float32), pr["ext"], rec[:, 2].astype(np.float32), cams,
                                 opts.tile)
    out = render(cams, opts, rec, ids, ranges)
    out.update(proj=pr, keys=keys, ids=ids, ranges=ranges)
    return out


def forward_backward_l1(params: Params, cams, targets, opts: Options):
    """Independent FP64 forward, L1 loss and gradient of every raw parameter."""
    f = forward(params, cams, opts)
    loss, dl = l1_loss(f["image"], targets, cams)
    g2 = render_backward(cams, opts, f["proj"]["rec"], f["ids"], f["ranges"], dl)
    grads = project_backward(params, cams, opts, g2)
    f.update(loss=loss, dl_dimage=dl, grad2d=g2, grads=grads)
    return f


PARAM_SLICES = ("means", 0, 3), ("log_scales", 3, 6), ("quats", 6, 10), ("opacity_logits", 10, 11)


def param_index_name(p: int):
    for name, a, b in PARAM_SLICES:
        if a <= p < b:
            return name, p - a
    return "sh", p - 11


def fd_local(params: Params, cams, targets, opts: Options, gauss_idx, param_idx, h_rel=1e-6):
    """Central finite differences of the L1 loss (see or_fd_local)."""
    g = np.ascontiguousarray(gauss_idx, np.int64)
    p = np.ascontiguousarray(param_idx, np.int32)
    out = np.zeros(g.shape[0])
    st = np.zeros(g.shape[0], np.int32)
    tgt = pack_views(targets)
    oc = opts.as_c()
    rc = lib().or_fd_local(params.n, params.sh_degree, _p(params.means), _p(params.log_scales), _p(params.quats),
                           _p(params.opacity_logits), _p(params.sh), cameras_c(cams), len(cams), C.byref(oc),
                           _p(tgt), g.shape[0], _p(g), _p(p), h_rel, _p(out), _p(st))
    assert rc == 0
    return out, st


def sh_basis(degree, dirs, with_grad=False):
    dirs = _d(dirs).reshape(-1, 3)
    n = dirs.shape[0]
    K = (degree + 1) ** 2
    Y = np.zeros((n, K))
    G = np.zeros((n, K, 3)) if with_grad else None
    lib().or_sh_basis(degree, n, _p(dirs), _p(Y), _p(G) if with_grad else None)
    return (Y, G) if with_grad else Y


def quat_to_rot(q_unit):
    q = _d(q_unit).reshape(4)
    R = np.zeros(9)
    lib().or_quat_to_rot(_p(q), _p(R))
    return R.reshape(3, 3)


# ---------------------------------------------------------------------------
# Adam (Kingma & Ba), with eps added to the bias-corrected root of the second
# moment; the 3DGS defaults adopted in Sec. IV-A: beta = (0.9, 0.999),
# eps = 1e-15, no weight decay, every element stepped.
# ---------------------------------------------------------------------------
def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One step in FP64; returns new (p, m, v).  `step` is the 1-based step count."""
    p, g, m, v = (np.asarray(x, np.float64) for x in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    p = p - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v
