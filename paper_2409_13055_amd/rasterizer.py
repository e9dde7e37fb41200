"""Device-side driver of the mapping step built on the libgs C ABI.

PyTorch only provides device memory and the stream; every step of the
rasteriser and the optimiser runs in the HIP kernels of libgs.so:

  Rasterizer       buffers + the four hot-path calls (project, bin/sort,
                   forward, backward) for a fixed set of keyframe cameras;
  render / RasterizeGaussians
                   torch.autograd.Function around them (dL/dimage from the
                   caller's loss);
  FusedAdam        gs_adam_step over the six parameter groups;
  MappingStep      one full iteration of the mapping module (Sec. III-B:
                   render, L1 term of eq. (2), backward, Adam) over a batch
                   of keyframes, runnable eagerly or replayed from a HIP
                   graph; PerViewMappingStep runs the same kernels one view
                   at a time;
  PointCloudInit   a keyframe's tracked pixels triangulated (gs_delaunay),
                   depth interpolated over low-gradient pixels and new
                   Gaussians initialised from it (Sec. III-A, III-B);
  ImagePyramid / PyramidMappingStep
                   the Gaussian pyramid of the ground-truth images
                   (gs_pyramid_reduce, Sec. III-B) and coarse-to-fine
                   mapping over its levels with one shared Adam state.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest")


def _p(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class GaussianParams:
    """The Gaussian set of Sec. III-B as six FP32 device tensors."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh_dc, sh_rest, sh_degree: int):
        self.means, self.log_scales, self.quats = means, log_scales, quats
        self.opacity_logits, self.sh_dc, self.sh_rest = opacity_logits, sh_dc, sh_rest
        self.sh_degree = int(sh_degree)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_scene(scene, device="cuda") -> "GaussianParams":
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device).contiguous()  # noqa: E731
        return GaussianParams(f(scene.means), f(scene.log_scales), f(scene.quats), f(scene.opacity_logits),
                              f(scene.sh_dc), f(scene.sh_rest), scene.sh_degree)

    @staticmethod
    def empty(n: int, sh_degree: int, device="cuda") -> "GaussianParams":
        K = (sh_degree + 1) ** 2
        e = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=device)  # noqa: E731
        return GaussianParams(e(n, 3), e(n, 3), e(n, 4), e(n), e(n, 3), e(n, K - 1, 3), sh_degree)

    def tensors(self) -> List[torch.Tensor]:
        return [getattr(self, k) for k in PARAM_NAMES]

    def zeros_like(self) -> "GaussianParams":
        return GaussianParams(*[torch.zeros_like(t) for t in self.tensors()], self.sh_degree)

    def c_params(self) -> L.gs_params:
        p = L.gs_params()
        p.n, p.sh_degree = self.n, self.sh_degree
        p.means, p.log_scales, p.quats = _p(self.means), _p(self.log_scales), _p(self.quats)
        p.opacity_logits, p.sh_dc = _p(self.opacity_logits), _p(self.sh_dc)
        p.sh_rest = _p(self.sh_rest) if self.sh_degree > 0 else None
        return p

    def c_grads(self) -> L.gs_grads:
        g = L.gs_grads()
        g.means, g.log_scales, g.quats = _p(self.means), _p(self.log_scales), _p(self.quats)
        g.opacity_logits, g.sh_dc = _p(self.opacity_logits), _p(self.sh_dc)
        g.sh_rest = _p(self.sh_rest) if self.sh_degree > 0 else None
        return g

    def spatial_order(self) -> torch.Tensor:
        """gs_spatial_order: the permutation (int32 [n], position k <- Gaussian order[k]) that sorts the
        set by the Morton code of the means.  Enqueued on the current stream."""
        ws = torch.empty(L.gs_spatial_order_workspace_size(self.n), dtype=torch.uint8, device=self.means.device)
        order = torch.empty(self.n, dtype=torch.int32, device=self.means.device)
        L.gs_spatial_order(_p(self.means), self.n, _p(order), _p(ws), ws.numel(), _stream())
        return order

    def gathered(self, order: torch.Tensor) -> "GaussianParams":
        """A new set with row k = row order[k] of this one (gs_gather_rows on every array)."""
        return GaussianParams(*[gather_rows(t, order) for t in self.tensors()], self.sh_degree)


def gather_rows(t: torch.Tensor, order: torch.Tensor) -> torch.Tensor:
    """gs_gather_rows: out[k] = t[order[k]] for a contiguous FP32 tensor of n rows."""
    n = int(t.shape[0])
    out = torch.empty_like(t)
    width = t.numel() // n if n else 0
    if n and width:
        L.gs_gather_rows(_p(t.contiguous()), n, width, _p(order), _p(out), _stream())
    return out


def pack_images(images: Sequence, device="cuda") -> torch.Tensor:
    """Per-view [3,H,W] images -> one packed FP32 device buffer (view-major, planar)."""
    parts = [torch.as_tensor(np.ascontiguousarray(a, np.float32)).reshape(-1) for a in images]
    return torch.cat(parts).to(device).contiguous()


def unpack_images(flat: torch.Tensor, cameras, channels=3) -> List[torch.Tensor]:
    out, off = [], 0
    for c in cameras:
        k = channels * c.width * c.height
        a = flat[off:off + k]
        out.append(a.view(channels, c.height, c.width) if channels > 1 else a.view(c.height, c.width))
        off += k
    return out


class Frame:
    """Buffers of one rendered batch: projected records, bins, image.  The bins are tile lists
    (ids, ranges) or window lists (items, win_ranges), as the rasteriser's `lists` says."""

    def __init__(self, rast: "Rasterizer", capacity: int):
        dev = rast.device
        VN = rast.n * rast.n_views
        self.windowed = rast.lists == "window"
        self.rec = torch.empty(VN * L.GS_REC_FLOATS, dtype=torch.float32, device=dev)
        self.tiles = torch.empty(VN, dtype=torch.int32, device=dev)
        n_seg = rast.n_views * ((rast.n + 63) // 64)  # visible pairs by (view, 64 Gaussians), see gs_projected
        self.vis = torch.empty(n_seg * 64 * 4, dtype=torch.int32, device=dev)
        self.vis_count = torch.empty(n_seg, dtype=torch.int32, device=dev)
        # the ranges start empty, so a raster call before any sort reads no list
        if self.windowed:
            self.ranges = None
            self.win_ranges = torch.zeros(2 * max(1, rast.total_windows), dtype=torch.int32, device=dev)
        else:
            self.ranges = torch.zeros(2 * rast.total_tiles, dtype=torch.int32, device=dev)
            self.win_ranges = None
        self.d_num_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
        self.d_num_items = torch.zeros(1, dtype=torch.int64, device=dev)
        self.d_overflow = torch.zeros(1, dtype=torch.int32, device=dev)
        self.rgb = torch.empty(3 * rast.total_pixels, dtype=torch.float32, device=dev)
        if rast.checkpoint:
            self.t_final = self.n_contrib = None
        else:
            self.t_final = torch.empty(rast.total_pixels, dtype=torch.float32, device=dev)
            self.n_contrib = torch.empty(rast.total_pixels, dtype=torch.int32, device=dev)
        self.keys = None
        self.set_capacity(capacity, rast.want_keys)

    def set_capacity(self, capacity: int, want_keys: bool):
        """Buffers for `capacity` list entries: incidences of the tile lists, or items of the window
        lists (8 bytes each: the pair and its clipped rect)."""
        dev = self.rec.device
        self.capacity = int(capacity)
        if self.windowed:
            self.ids = self.keys = None
            self.items = torch.empty(max(1, self.capacity), dtype=torch.int64, device=dev)
        else:
            self.items = None
            self.ids = torch.empty(max(1, self.capacity), dtype=torch.int32, device=dev)
            self.keys = torch.empty(max(1, self.capacity), dtype=torch.int64, device=dev) if want_keys else None

    def c_proj(self) -> L.gs_projected:
        return L.gs_projected(_p(self.rec), _p(self.tiles), _p(self.vis), _p(self.vis_count))

    def c_bins(self) -> L.gs_bins:
        b = L.gs_bins()
        b.keys, b.ids, b.ranges = _p(self.keys), _p(self.ids), _p(self.ranges)
        b.items, b.win_ranges, b.d_num_items = _p(self.items), _p(self.win_ranges), _p(self.d_num_items)
        b.capacity = self.capacity
        b.d_num_pairs, b.d_overflow = _p(self.d_num_pairs), _p(self.d_overflow)
        return b

    def list_entries(self) -> int:
        """The entries the bins hold after gs_bin_sort (syncs): window items or tile incidences."""
        return int((self.d_num_items if self.windowed else self.d_num_pairs).item())

    def c_image(self) -> L.gs_image:
        return L.gs_image(_p(self.rgb), _p(self.t_final), _p(self.n_contrib))


class Rasterizer:
    """The four rasteriser calls of libgs for a fixed set of keyframe cameras.  lists: the form of
    the bins, "window" (gs_bin_sort writes each 8 x 8-tile window's list and the raster kernels take
    a tile's entries from it; the default, it skips writing the tile lists) or "tile" (the tile
    lists and ranges, which `want_keys` extends with the sort keys)."""

    def __init__(self, cameras, n: int, sh_degree: int, tile_size: int = 16, checkpoint: bool = False,
                 device="cuda", want_keys: bool = False, growth: float = 1.25, lists: str = "window",
                 **opt_overrides):
        L.load()
        if lists not in ("window", "tile"):
            raise ValueError(f"lists must be 'window' or 'tile', not {lists!r}")
        if want_keys and lists != "tile":
            raise ValueError("the sort keys come with tile lists (lists='tile')")
        self.lists = lists
        self.cameras = list(cameras)
        self.n_views = len(self.cameras)
        self.n = int(n)
        self.sh_degree = int(sh_degree)
        self.device = torch.device(device)
        self.checkpoint = bool(checkpoint)
        self.want_keys = want_keys
        self.growth = growth
        self.opts = L.default_options(tile_size=int(tile_size), checkpoint=int(checkpoint), **opt_overrides)
        if lists == "window":
            self.opts.flags |= L.GS_OPT_WINDOW_LISTS
        self.cams = L.make_cameras(self.cameras)
        self.total_tiles = L.gs_total_tiles(self.cams, self.n_views, self.opts.tile_size)
        self.total_windows = L.gs_total_windows(self.cams, self.n_views, self.opts.tile_size)
        self.total_pixels = L.gs_total_pixels(self.cams, self.n_views)
        self.capacity = 0
        self.ws_sort = None
        self.ws_sort_bytes = 0
        self.ws_fwd_bytes = L.gs_render_fwd_workspace_size(self.cams, self.n_views, self.opts)
        self.ws_fwd = torch.empty(self.ws_fwd_bytes, dtype=torch.uint8, device=self.device)
        self.ws_bwd_bytes = L.gs_render_bwd_workspace_size(self.n, self.n_views)
        self.ws_bwd = torch.empty(self.ws_bwd_bytes, dtype=torch.uint8, device=self.device)
        self._ensure_sort_ws(0)

    def _ensure_sort_ws(self, capacity: int):
        need = L.gs_bin_sort_workspace_size(self.n, self.cams, self.n_views, self.opts, capacity)
        if self.ws_sort is None or need > self.ws_sort_bytes:
            self.ws_sort = torch.empty(need, dtype=torch.uint8, device=self.device)
            self.ws_sort_bytes = need

    def reserve(self, capacity: int):
        """Set the list capacity used by new frames (tile incidences or window items; and grow the sort
        workspace)."""
        self.capacity = int(capacity)
        self._ensure_sort_ws(self.capacity)

    def new_frame(self) -> Frame:
        return Frame(self, self.capacity)

    # hot-path calls --------------------------------------------------------
    def project(self, params: GaussianParams, fr: Frame):
        L.gs_project(params.c_params(), self.cams, self.n_views, self.opts, fr.c_proj(), _stream())

    def bin_sort(self, fr: Frame):
        if fr.capacity != self.capacity:
            fr.set_capacity(self.capacity, self.want_keys)
        L.gs_bin_sort(fr.c_proj(), self.n, self.cams, self.n_views, self.opts, fr.c_bins(), self.ws_sort.data_ptr(),
                      self.ws_sort_bytes, _stream())

    def render_fwd(self, fr: Frame, target: Optional[torch.Tensor] = None, loss_out: Optional[torch.Tensor] = None):
        loss = L.gs_loss()
        if target is not None and loss_out is not None:
            loss.kind, loss.target, loss.loss_out = L.GS_LOSS_L1, _p(target), _p(loss_out)
        L.gs_render_fwd(fr.c_proj(), self.n, fr.c_bins(), self.cams, self.n_views, self.opts, loss, fr.c_image(),
                        self.ws_fwd.data_ptr(), self.ws_fwd_bytes, _stream())

    def render_bwd(self, params: GaussianParams, fr: Frame, grads: GaussianParams,
                   target: Optional[torch.Tensor] = None, dl_dimage: Optional[torch.Tensor] = None):
        loss = L.gs_loss()
        if dl_dimage is not None:
            loss.kind, loss.dl_dimage = L.GS_LOSS_EXTERNAL, _p(dl_dimage)
        else:
            loss.kind, loss.target = L.GS_LOSS_L1, _p(target)
        L.gs_render_bwd(params.c_params(), fr.c_proj(), fr.c_bins(), fr.c_image(), self.cams, self.n_views,
                        self.opts, loss, grads.c_grads(), self.ws_bwd.data_ptr(), self.ws_bwd_bytes, _stream())

    def _loss(self, target=None, dl_dimage=None) -> L.gs_loss:
        loss = L.gs_loss()
        if dl_dimage is not None:
            loss.kind, loss.dl_dimage = L.GS_LOSS_EXTERNAL, _p(dl_dimage)
        else:
            loss.kind, loss.target = L.GS_LOSS_L1, _p(target)
        return loss

    def raster_bwd(self, fr: Frame, grad2d: torch.Tensor, target=None, dl_dimage=None,
                   abs2d: Optional[torch.Tensor] = None):
        """Adds the image-space gradients of this frame into grad2d ([n_views*n, 9] FP32), and with
        abs2d ([n_views*n, 2]) the homodirectional view-space gradient (gs_raster_bwd_abs)."""
        if abs2d is None:
            L.gs_raster_bwd(fr.c_proj(), self.n, fr.c_bins(), fr.c_image(), self.cams, self.n_views, self.opts,
                            self._loss(target, dl_dimage), grad2d.data_ptr(), _stream())
        else:
            L.gs_raster_bwd_abs(fr.c_proj(), self.n, fr.c_bins(), fr.c_image(), self.cams, self.n_views, self.opts,
                                self._loss(target, dl_dimage), grad2d.data_ptr(), abs2d.data_ptr(), _stream())

    def project_bwd(self, params: GaussianParams, fr: Frame, grad2d: torch.Tensor, grads: GaussianParams):
        """Adds the parameter gradients chained from grad2d into grads."""
        L.gs_project_bwd(params.c_params(), fr.c_proj(), self.cams, self.n_views, self.opts, grad2d.data_ptr(),
                         grads.c_grads(), _stream())

    def project_bwd_adam(self, params: GaussianParams, fr: Frame, grad2d: torch.Tensor, adam: "FusedAdam",
                         density: Optional["DensityControl"] = None, abs2d: Optional[torch.Tensor] = None):
        """The projection backward of grad2d fused with adam's step (params and moments updated in place);
        with `density` and abs2d it also adds the iteration's density-control statistics
        (gs_project_bwd_adam_stats)."""
        if density is None:
            L.gs_project_bwd_adam(params.c_params(), fr.c_proj(), self.cams, self.n_views, self.opts,
                                  grad2d.data_ptr(), adam.all_groups, adam.betas[0], adam.betas[1], adam.eps,
                                  _p(adam.d_step), _stream())
        else:
            L.gs_project_bwd_adam_stats(params.c_params(), fr.c_proj(), self.cams, self.n_views, self.opts,
                                        grad2d.data_ptr(), adam.all_groups, adam.betas[0], adam.betas[1], adam.eps,
                                        _p(adam.d_step), _p(abs2d), density._stats, _stream())

    def render_stats(self, fr: Frame, out: Optional[torch.Tensor] = None) -> Optional[Dict[str, int]]:
        """Work counts of the blending of this frame (see gs_render_stats).  Without `out` it syncs
        and returns them; with `out` (3 int64 on the device) it only enqueues the count into it."""
        dst = torch.zeros(3, dtype=torch.int64, device=self.device) if out is None else out
        L.gs_render_stats(fr.c_proj(), self.n, fr.c_bins(), self.cams, self.n_views, self.opts, dst.data_ptr(),
                          _stream())
        if out is not None:
            return None
        e, b, c = (int(x) for x in dst.cpu())
        return {"evaluated": e, "blended": b, "contrib_prefix": c}

    @property
    def grad2d(self) -> torch.Tensor:
        """[n_views*n, 9] image-space gradients of the last backward."""
        return self.ws_bwd.view(torch.float32)[: self.n_views * self.n * 9].view(-1, 9)

    # eager helpers -----------------------------------------------------------
    def fit_capacity(self, fr: Frame) -> bool:
        """After bin_sort: if the pairs overflowed, grow the capacity and sort again (syncs)."""
        if int(fr.d_overflow.item()) == 0:
            return False
        m = fr.list_entries()
        self.reserve(int(math.ceil(m * self.growth)) + 1024)
        self.bin_sort(fr)
        assert int(fr.d_overflow.item()) == 0
        return True

    def forward(self, params: GaussianParams, fr: Optional[Frame] = None, target=None, loss_out=None) -> Frame:
        fr = fr or self.new_frame()
        self.project(params, fr)
        self.bin_sort(fr)
        self.fit_capacity(fr)
        self.render_fwd(fr, target, loss_out)
        return fr


class RasterizeGaussians(torch.autograd.Function):
    """image = render(Gaussians); backward takes dL/dimage from the caller's loss."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, means, log_scales, quats, opacity_logits, sh_dc, sh_rest):
        params = GaussianParams(means.contiguous(), log_scales.contiguous(), quats.contiguous(),
                                opacity_logits.contiguous(), sh_dc.contiguous(), sh_rest.contiguous(),
                                rast.sh_degree)
        fr = rast.forward(params)
        ctx.rast, ctx.frame, ctx.params = rast, fr, params
        return fr.rgb.clone()

    @staticmethod
    def backward(ctx, dl_dimage):
        grads = ctx.params.zeros_like()
        ctx.rast.render_bwd(ctx.params, ctx.frame, grads, dl_dimage=dl_dimage.contiguous())
        return (None, *grads.tensors())


def render(rast: Rasterizer, means, log_scales, quats, opacity_logits, sh_dc, sh_rest) -> torch.Tensor:
    """Differentiable render of all views of `rast`; returns the packed [sum 3HW] image."""
    return RasterizeGaussians.apply(rast, means, log_scales, quats, opacity_logits, sh_dc, sh_rest)


class PhotometricLoss:
    """eq. (2) with its SSIM term for a fixed set of keyframes (gs_photometric_loss): per view
    (1 - lam) L1 + lam (1 - SSIM), and dL/dimage for the raster backward."""

    def __init__(self, cameras, device="cuda"):
        L.load()
        self.cams = L.make_cameras(list(cameras))
        self.n_views = len(cameras)
        self.ws_bytes = L.gs_photometric_loss_workspace_size(self.cams, self.n_views)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def __call__(self, image: torch.Tensor, target: torch.Tensor, lam: float,
                 loss_out: Optional[torch.Tensor] = None, dl_dimage: Optional[torch.Tensor] = None):
        L.gs_photometric_loss(self.cams, self.n_views, _p(image), _p(target), float(lam), _p(loss_out),
                              _p(dl_dimage), self.ws.data_ptr(), self.ws_bytes, _stream())


class FusedAdam:
    """Adam over the six parameter groups in one gs_adam_step launch (step counter on the device)."""

    def __init__(self, params: GaussianParams, grads: GaussianParams, lrs: Dict[str, float],
                 betas=(0.9, 0.999), eps=1e-15, exp_avg: Optional[GaussianParams] = None,
                 exp_avg_sq: Optional[GaussianParams] = None, d_step: Optional[torch.Tensor] = None):
        """exp_avg, exp_avg_sq, d_step: an existing optimiser state to continue (density control
        hands over the moments of the new Gaussian set); None starts from zero."""
        self.params, self.grads = params, grads
        self.lrs = dict(lrs)
        self.exp_avg = exp_avg if exp_avg is not None else params.zeros_like()
        self.exp_avg_sq = exp_avg_sq if exp_avg_sq is not None else params.zeros_like()
        self.betas, self.eps = betas, eps
        self.d_step = d_step if d_step is not None else torch.zeros(1, dtype=torch.int32, device=params.means.device)
        names = [k for k in PARAM_NAMES if getattr(params, k).numel() > 0]
        self.groups = (L.gs_adam_group * len(names))()
        for i, k in enumerate(names):
            g = self.groups[i]
            g.param, g.grad = _p(getattr(params, k)), _p(getattr(grads, k))
            g.exp_avg, g.exp_avg_sq = _p(getattr(self.exp_avg, k)), _p(getattr(self.exp_avg_sq, k))
            g.numel, g.lr = getattr(params, k).numel(), float(lrs[k])
        self.n_groups = len(names)
        # all six groups in parameter order, for the projection backward fused with the step
        self.all_groups = (L.gs_adam_group * len(PARAM_NAMES))()
        for i, k in enumerate(PARAM_NAMES):
            g = self.all_groups[i]
            t = getattr(params, k)
            if t.numel() > 0:
                g.param = _p(t)
                g.exp_avg, g.exp_avg_sq = _p(getattr(self.exp_avg, k)), _p(getattr(self.exp_avg_sq, k))
            g.numel, g.lr = t.numel(), float(lrs[k])

    def step(self, zero_grad: bool = True):
        L.gs_adam_step(self.groups, self.n_groups, self.betas[0], self.betas[1], self.eps, _p(self.d_step),
                       1 if zero_grad else 0, _stream())

    def gathered(self, params: GaussianParams, order: torch.Tensor) -> "FusedAdam":
        """The optimiser over `params` (this optimiser's set reordered by `order`, see
        GaussianParams.gathered) with the moments reordered the same way and the step count kept."""
        return FusedAdam(params, self.grads.gathered(order), self.lrs, self.betas, self.eps,
                         exp_avg=self.exp_avg.gathered(order), exp_avg_sq=self.exp_avg_sq.gathered(order),
                         d_step=self.d_step.clone())


def spatially_ordered(params: GaussianParams, adam: Optional[FusedAdam] = None):
    """The Gaussian set (and its optimiser, when given) reordered by gs_spatial_order: a memory layout
    that lets the projection and its backward skip the views a wavefront's 64 Gaussians are all
    outside of.  Returns (params, adam, order); the set is the same, only its order changes."""
    order = params.spatial_order()
    new_p = params.gathered(order)
    return new_p, (adam.gathered(new_p, order) if adam is not None else None), order


class CapacityOverflow(RuntimeError):
    """The pair capacity of a captured or repeated iteration was exceeded."""


class MappingStep:
    """One mapping iteration over a batch of keyframes (Sec. III-B): project all
    views in one pass over the parameters, one bin/sort over every view's
    tiles, forward with the fused L1 loss, backward, and optionally Adam.  With
    fuse_adam (the default when Adam is on) the projection backward applies the
    Adam step itself, so the raw-parameter gradients never reach memory;
    otherwise the gradients are accumulated into `grads` and Adam (which also
    clears them) runs as its own call."""

    def __init__(self, params: GaussianParams, cameras, targets, lrs=None, tile_size=16, checkpoint=False,
                 with_adam=True, fuse_adam=True, ssim_lambda: float = 0.0, adam: Optional[FusedAdam] = None,
                 density: Optional["DensityControl"] = None, **opt):
        """`adam`: an existing FusedAdam over `params` to step (steps that train the same Gaussians on
        other views or pyramid levels share its moments and step count); None makes a new one.
        `density`: a DensityControl whose statistics every iteration adds to (the raster backward then
        also forms the homodirectional gradient); densify() hands over to a step on the new set."""
        self.params = params
        self.density = density
        self._init = dict(cameras=list(cameras), lrs=lrs, tile_size=tile_size, checkpoint=checkpoint,
                          with_adam=with_adam, fuse_adam=fuse_adam, ssim_lambda=ssim_lambda, opt=dict(opt))
        if density is not None and not (with_adam and fuse_adam):
            raise ValueError("density control runs with the fused projection backward and Adam")
        # eq. (2): with ssim_lambda > 0 the loss is (1 - lambda) L1 + lambda (1 - SSIM) (3DGS: 0.2),
        # computed by gs_photometric_loss after the forward; 0 keeps the L1 term fused into the forward
        self.ssim_lambda = float(ssim_lambda)
        self.fuse_adam = with_adam and fuse_adam
        self.rast = Rasterizer(cameras, params.n, params.sh_degree, tile_size=tile_size, checkpoint=checkpoint,
                               device=params.means.device, **opt)
        if adam is not None and (not with_adam or adam.params is not params):
            raise ValueError("a shared FusedAdam must step the same parameters, with with_adam=True")
        self.grads = adam.grads if adam is not None else params.zeros_like()
        self.target = targets if isinstance(targets, torch.Tensor) else pack_images(targets, params.means.device)
        self.loss = torch.zeros(self.rast.n_views, dtype=torch.float32, device=params.means.device)
        self.adam = adam if adam is not None else (FusedAdam(params, self.grads, lrs) if with_adam else None)
        self.photometric = None
        self.dl_dimage = None
        if self.ssim_lambda > 0.0:
            self.photometric = PhotometricLoss(cameras, device=params.means.device)
            self.dl_dimage = torch.empty(3 * self.rast.total_pixels, dtype=torch.float32, device=params.means.device)
        self.frame = None
        self.graph = None
        self._side = None  # stream of the gradient-buffer clear, which overlaps the forward
        # 1 once any iteration since the last check_overflow() overflowed the pair capacity (that
        # iteration rendered nothing: gs_bin_sort leaves every tile empty); set on the device, so
        # graph replays keep it too
        self.overflow_seen = torch.zeros(1, dtype=torch.int32, device=params.means.device)
        self.abs2d = None
        if density is not None:
            self.abs2d = torch.empty(self.rast.n_views * params.n, 2, dtype=torch.float32, device=params.means.device)

    def size(self):
        """Eager warm-up that sizes the pair capacity (host syncs)."""
        fr = self.frame or self.rast.new_frame()
        self.rast.project(self.params, fr)
        self.rast.bin_sort(fr)
        self.rast.fit_capacity(fr)
        self.frame = fr

    def _forward(self, fr, mark=None):
        """Forward raster and the loss: L1 fused into the forward, or eq. (2) with SSIM after it."""
        r = self.rast
        if self.photometric is None:
            r.render_fwd(fr, self.target, self.loss)
            if mark:
                mark("render_fwd")
            return
        r.render_fwd(fr)
        if mark:
            mark("render_fwd")
        self.photometric(fr.rgb, self.target, self.ssim_lambda, self.loss, self.dl_dimage)
        if mark:
            mark("photometric_loss")

    def _loss_args(self):
        return dict(target=self.target) if self.photometric is None else dict(dl_dimage=self.dl_dimage)

    def run(self, mark=None):
        """Enqueue one iteration (no host synchronisation); see _run.  The iteration's overflow flag
        is folded into overflow_seen after its last stage."""
        self._run(mark)
        torch.maximum(self.overflow_seen, self.frame.d_overflow, out=self.overflow_seen)

    def _run(self, mark=None):
        """Enqueue one iteration (no host synchronisation).

        With `mark` (a callable taking a stage name), the backward is issued as
        its two calls (raster backward into the image-space gradient buffer,
        then the projection backward) and mark(name) is called on the host after
        each stage is enqueued, so a caller can record stream events between
        the stages of an iteration."""
        r, fr = self.rast, self.frame
        r.project(self.params, fr)
        if mark:
            mark("project")
        r.bin_sort(fr)
        if mark:
            mark("bin_sort")
        if self.fuse_adam and mark is None:
            # The image-space gradient buffer is cleared on a second stream while the forward runs:
            # the fill is bound by memory bandwidth, the forward by ALU issue.  The previous
            # iteration's reader of the buffer precedes the fork in stream order.
            cur = torch.cuda.current_stream()
            if self._side is None:
                self._side = torch.cuda.Stream(device=cur.device)
            self._side.wait_stream(cur)
            with torch.cuda.stream(self._side):
                r.grad2d.zero_()
                if self.abs2d is not None:
                    self.abs2d.zero_()
            self._forward(fr)
            cur.wait_stream(self._side)
            r.raster_bwd(fr, r.grad2d, abs2d=self.abs2d, **self._loss_args())
            r.project_bwd_adam(self.params, fr, r.grad2d, self.adam, density=self.density, abs2d=self.abs2d)
            return
        self._forward(fr, mark)
        if self.fuse_adam:
            g2 = r.grad2d
            g2.zero_()
            if self.abs2d is not None:
                self.abs2d.zero_()
            if mark:
                mark("clear_grad2d")
            r.raster_bwd(fr, g2, abs2d=self.abs2d, **self._loss_args())
            if mark:
                mark("raster_bwd")
            r.project_bwd_adam(self.params, fr, g2, self.adam, density=self.density, abs2d=self.abs2d)
            if mark:
                mark("project_bwd_adam")
            return
        if mark is None:
            r.render_bwd(self.params, fr, self.grads, **self._loss_args())
        else:
            g2 = r.grad2d
            g2.zero_()
            mark("clear_grad2d")
            r.raster_bwd(fr, g2, **self._loss_args())
            mark("raster_bwd")
            r.project_bwd(self.params, fr, g2, self.grads)
            mark("project_bwd")
        if self.adam is not None:
            self.adam.step(zero_grad=True)
            if mark:
                mark("adam")

    def overflowed(self) -> bool:
        return int(self.frame.d_overflow.item()) != 0

    def check_overflow(self):
        """Raises CapacityOverflow when an iteration since the last check overflowed the pair capacity
        (synchronises with the host); the flag is cleared."""
        if int(self.overflow_seen.item()) != 0:
            self.overflow_seen.zero_()
            raise CapacityOverflow(f"the list entries (tile incidences or window items) exceeded the capacity "
                                   f"{self.rast.capacity}: "
                                   f"those iterations rendered empty tiles and stepped Adam on zero gradients; "
                                   f"size() again (and capture()) before continuing")

    def densify(self, generator: Optional[torch.Generator] = None) -> "MappingStep":
        """One density-control step (Sec. III-B) on this step's Gaussians; returns a MappingStep over
        the new set, sized, with the optimiser state handed over (a captured graph is not carried:
        capture() again).  Synchronises with the host (the new size is read back)."""
        new_params, new_adam = self.density.apply(self.params, self.adam, generator=generator)
        k = self._init
        st = MappingStep(new_params, k["cameras"], self.target, lrs=k["lrs"], tile_size=k["tile_size"],
                         checkpoint=k["checkpoint"], with_adam=k["with_adam"], fuse_adam=k["fuse_adam"],
                         ssim_lambda=k["ssim_lambda"], adam=new_adam, density=self.density, **k["opt"])
        st.size()
        return st

    def capture(self):
        """Record one iteration into a HIP graph (after size())."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()  # one eager iteration on the capture stream before recording
        torch.cuda.current_stream().wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()

    def replay(self):
        self.graph.replay()


class PerViewMappingStep:
    """The same iteration with every keyframe rendered by its own calls
    (projection re-reads the parameters per view; gradients accumulate)."""

    def __init__(self, params: GaussianParams, cameras, targets, lrs=None, tile_size=16, checkpoint=False,
                 with_adam=True, **opt):
        self.params = params
        dev = params.means.device
        self.rasts = [Rasterizer([c], params.n, params.sh_degree, tile_size=tile_size, checkpoint=checkpoint,
                                 device=dev, **opt) for c in cameras]
        self.grads = params.zeros_like()
        self.targets = [pack_images([t], dev) for t in targets]
        self.losses = [torch.zeros(1, dtype=torch.float32, device=dev) for _ in cameras]
        self.adam = FusedAdam(params, self.grads, lrs) if with_adam else None
        self.frames = [None] * len(cameras)
        self.graph = None

    def size(self):
        for k, r in enumerate(self.rasts):
            fr = self.frames[k] or r.new_frame()
            r.project(self.params, fr)
            r.bin_sort(fr)
            r.fit_capacity(fr)
            self.frames[k] = fr

    def run(self):
        for r, fr, tg, ls in zip(self.rasts, self.frames, self.targets, self.losses):
            r.project(self.params, fr)
            r.bin_sort(fr)
            r.render_fwd(fr, tg, ls)
            r.render_bwd(self.params, fr, self.grads, target=tg)
        if self.adam is not None:
            self.adam.step(zero_grad=True)

    def overflowed(self) -> bool:
        return any(int(fr.d_overflow.item()) != 0 for fr in self.frames)

    def capture(self):
        """Record one iteration (every view's calls, then Adam) into a HIP graph (after size())."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()

    def replay(self):
        self.graph.replay()


@dataclasses.dataclass
class LevelCamera:
    """A keyframe camera as gs_camera holds it (R row-major, world to camera)."""
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


def pyramid_camera(cam, levels: int) -> LevelCamera:
    """The camera that samples `levels` pyramid reductions of cam's image (gs_pyramid_camera)."""
    c = L.gs_pyramid_camera(L.make_cameras([cam])[0], int(levels))
    return LevelCamera(np.array(c.R[:], np.float64).reshape(3, 3), np.array(c.t[:], np.float64), c.fx, c.fy, c.cx,
                       c.cy, c.width, c.height)


class ImagePyramid:
    """Gaussian pyramid of the keyframes' ground-truth images (Sec. III-B): level 0 is the packed
    input, level l + 1 one gs_pyramid_reduce of level l for all views at once; cameras[l] samples
    level l."""

    def __init__(self, cameras, images, levels: int, device="cuda"):
        if levels < 0:
            raise ValueError("levels must be >= 0")
        L.load()
        base = images if isinstance(images, torch.Tensor) else pack_images(images, device)
        self.cameras = [list(cameras)]
        self.images = [base]
        self._c_cams = []  # host gs_camera arrays of the levels that are reduced
        for _ in range(levels):
            src_cams = self.cameras[-1]
            dst_cams = [pyramid_camera(c, 1) for c in src_cams]
            self._c_cams.append(L.make_cameras(src_cams))
            self.cameras.append(dst_cams)
            self.images.append(torch.empty(sum(3 * c.width * c.height for c in dst_cams), dtype=torch.float32,
                                           device=base.device))
            self.reduce_level(len(self.images) - 2)

    def reduce_level(self, level: int):
        """Recompute level + 1 from level (one gs_pyramid_reduce over all views)."""
        src_cams = self._c_cams[level]
        L.gs_pyramid_reduce(src_cams, len(src_cams), _p(self.images[level]), _p(self.images[level + 1]), _stream())

    @staticmethod
    def reduce(cams, src: torch.Tensor, dst: torch.Tensor):
        """dst = one pyramid level of the packed views src (cameras `cams` of src)."""
        L.gs_pyramid_reduce(L.make_cameras(list(cams)), len(cams), _p(src), _p(dst), _stream())

    @property
    def levels(self) -> int:
        return len(self.images) - 1

    def view(self, level: int, v: int) -> torch.Tensor:
        """The slice of level `level` holding view v ([3 H W], planar)."""
        cams = self.cameras[level]
        off = sum(3 * c.width * c.height for c in cams[:v])
        return self.images[level][off:off + 3 * cams[v].width * cams[v].height]

    def batch(self, view_levels: Sequence[int]):
        """Cameras and packed targets of a batch whose view v is taken at level view_levels[v]."""
        cams = [self.cameras[l][v] for v, l in enumerate(view_levels)]
        if all(l == view_levels[0] for l in view_levels):
            return cams, self.images[view_levels[0]]
        return cams, torch.cat([self.view(l, v) for v, l in enumerate(view_levels)])


class PyramidMappingStep:
    """Coarse-to-fine mapping (Sec. III-B, after Photo-SLAM): the loss of the first iterations uses
    the coarsest pyramid level of the ground-truth images, later ones finer levels.

    `schedule[k]` iterations run at level levels - k (k = 0 the coarsest), after which every
    iteration runs at level 0.  Each batch of per-view levels gets its own MappingStep (its own
    buffers and, after capture(), its own HIP graph); all of them step the same Gaussians with one
    FusedAdam, so the moments and the step count carry across levels.  run_levels() takes an
    explicit per-view level tuple: keyframes at different levels share one batch."""

    def __init__(self, params: GaussianParams, cameras, targets, levels: int = 2, schedule=None, lrs=None,
                 graphs: bool = True, adam: Optional[FusedAdam] = None, pyramid: Optional["ImagePyramid"] = None,
                 iteration: int = 0, autotune: bool = False, **step_opts):
        """`adam`, `pyramid`, `iteration`: an optimiser state, a built pyramid of these targets and a
        position in the schedule to continue from (after density control changed the set).
        autotune: each batch of per-view levels takes the tile size, LDS batch and bins form that
        gs_autotune picks for it (coarse levels favour other settings than full resolution), in
        place of those in step_opts."""
        self.params = params
        self.pyramid = pyramid if pyramid is not None else ImagePyramid(cameras, targets, levels,
                                                                        device=params.means.device)
        levels = self.pyramid.levels
        self.schedule = list(schedule) if schedule is not None else [100] * levels
        if len(self.schedule) != levels:
            raise ValueError("schedule needs one iteration count per coarse level")
        self.n_views = len(cameras)
        self.lrs = lrs
        self.graphs = graphs
        self.step_opts = step_opts
        self.autotune = bool(autotune)
        self.tuned: Dict[tuple, dict] = {}  # per level batch: what the autotuner chose
        self.adam = adam if adam is not None else FusedAdam(params, params.zeros_like(), lrs)
        self.steps: Dict[tuple, MappingStep] = {}
        self._ran_at_capture = set()  # keys whose newest iteration capture() already ran
        self.iteration = int(iteration)

    def level_at(self, iteration: int) -> int:
        lv = self.pyramid.levels
        for k, n in enumerate(self.schedule):
            if iteration < n:
                return lv - k
            iteration -= n
        return 0

    def step_for(self, view_levels: Sequence[int]) -> MappingStep:
        key = tuple(int(l) for l in view_levels)
        if len(key) != self.n_views or any(l < 0 or l > self.pyramid.levels for l in key):
            raise ValueError(f"bad per-view levels {key}")
        st = self.steps.get(key)
        if st is None:
            cams, tgt = self.pyramid.batch(key)
            opts = dict(self.step_opts)
            if self.autotune:
                from .autotune import autotune_tile  # (the autotuner's binding imports this module)
                tune = autotune_tile(self.params, cams, tgt, checkpoint=bool(opts.get("checkpoint", False)), iters=2)
                opts.update(tile_size=tune["best"], lds_batch=tune["lds_batch"], lists=tune["lists"])
                self.tuned[key] = tune
            st = MappingStep(self.params, cams, tgt, lrs=self.lrs, adam=self.adam, **opts)
            st.size()
            if self.graphs:
                st.capture()  # runs one iteration eagerly, then records one
                self._ran_at_capture.add(key)
            self.steps[key] = st
        return st

    def run_levels(self, view_levels: Sequence[int]) -> MappingStep:
        """One iteration with view v at level view_levels[v]."""
        st = self.step_for(view_levels)
        key = tuple(int(l) for l in view_levels)
        if key in self._ran_at_capture:
            self._ran_at_capture.discard(key)
        elif st.graph is not None:
            st.replay()
        else:
            st.run()
        return st

    def run(self) -> MappingStep:
        """One iteration at the scheduled level (every view at the same level)."""
        st = self.run_levels([self.level_at(self.iteration)] * self.n_views)
        self.iteration += 1
        return st

    def check_overflow(self):
        """MappingStep.check_overflow of every level batch (synchronises)."""
        for st in self.steps.values():
            st.check_overflow()


class DensityControl:
    """Adaptive density control of Sec. III-B (AbsGS densification with the 3DGS split and clone
    parameters, pruning by opacity): per-Gaussian statistics that every iteration adds to
    (gs_density_accumulate), and the densify-and-prune step (gs_density_plan, then
    gs_density_apply into new arrays).  The paper runs the step every 1000 iterations (Sec. IV-A).

    `extent` defaults to the 3DGS scene extent of `cameras` (gs_scene_extent); other keyword
    arguments override gs_default_density_config (grad_threshold, percent_dense, min_opacity,
    split_scale_div)."""

    def __init__(self, n: int, cameras, device="cuda", extent: Optional[float] = None, **cfg):
        L.load()
        self.device = torch.device(device)
        cams = L.make_cameras(list(cameras))
        self.cfg = L.default_density_config(**cfg)
        self.cfg.extent = float(extent) if extent is not None else L.gs_scene_extent(cams, len(cameras))
        self.d_counts = torch.zeros(3, dtype=torch.int32, device=self.device)
        self._alloc(n)

    def _alloc(self, n: int):
        self.n = int(n)
        self.grad_accum = torch.zeros(self.n, dtype=torch.float32, device=self.device)
        self.abs_accum = torch.zeros(self.n, dtype=torch.float32, device=self.device)
        self.count = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        # an empty set (everything pruned) has no plan to hold
        self.ws_bytes = L.gs_density_workspace_size(self.n) if self.n > 0 else 0
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self._stats = L.gs_density_stats(_p(self.grad_accum), _p(self.abs_accum), _p(self.count))

    def accumulate(self, rast: Rasterizer, fr: Frame, grad2d: torch.Tensor, abs2d: torch.Tensor):
        L.gs_density_accumulate(fr.c_proj(), rast.n, rast.cams, rast.n_views, _p(grad2d), _p(abs2d), self._stats,
                                _stream())

    def plan_launch(self, params: GaussianParams):
        """Classify every Gaussian into the workspace and write the counts to d_counts (no sync)."""
        if params.n != self.n:
            raise ValueError("the statistics belong to a Gaussian set of another size")
        L.gs_density_plan(params.c_params(), self._stats, self.cfg, _p(self.d_counts), self.ws.data_ptr(),
                          self.ws_bytes, _stream())

    def plan(self, params: GaussianParams):
        """Classify (device) and return (kept, cloned, split) (host sync)."""
        self.plan_launch(params)
        kept, cloned, split = (int(x) for x in self.d_counts.cpu())
        return kept, cloned, split

    def apply_into(self, params: GaussianParams, adam: FusedAdam, eps: torch.Tensor, new_p: GaussianParams,
                   new_m: GaussianParams, new_v: GaussianParams):
        """gs_density_apply of the last plan into preallocated arrays of the new size."""
        L.gs_density_apply(params.c_params(), adam.exp_avg.c_params(), adam.exp_avg_sq.c_params(), self.cfg,
                           _p(eps), eps.numel(), new_p.n, new_p.c_grads(), new_m.c_grads(), new_v.c_grads(),
                           self.ws.data_ptr(), self.ws_bytes, _stream())

    def apply(self, params: GaussianParams, adam: FusedAdam, generator: Optional[torch.Generator] = None,
              eps: Optional[torch.Tensor] = None):
        """plan() then the new Gaussian set: returns (new params, FusedAdam over them continuing the
        step count).  The split children's standard normal draws are `eps` ([split, 2, 3]) or drawn
        with `generator`.  The statistics restart at zero for the new set."""
        kept, cloned, split = self.plan(params)
        n_out = kept + cloned + 2 * split
        if eps is None:
            eps = torch.randn(split, 2, 3, generator=generator, dtype=torch.float32, device=self.device)
        eps = eps.contiguous()
        D = params.sh_degree
        new_p = GaussianParams.empty(n_out, D, self.device)
        new_m = GaussianParams.empty(n_out, D, self.device)
        new_v = GaussianParams.empty(n_out, D, self.device)
        self.apply_into(params, adam, eps, new_p, new_m, new_v)
        self._alloc(n_out)
        new_adam = FusedAdam(new_p, new_p.zeros_like(), adam.lrs, adam.betas, adam.eps, exp_avg=new_m,
                             exp_avg_sq=new_v, d_step=adam.d_step)
        self.last_counts = (kept, cloned, split)
        return new_p, new_adam


class PointCloudInit:
    """New Gaussians for a keyframe (Sec. III-A, III-B): its tracked pixels (integer xy, depth) are
    triangulated on the host (gs_delaunay), the pixels of low-gradient regions take the mean depth of
    their triangle's vertices (gs_densify_depth), and one Gaussian starts at every pixel with a depth
    on the stride grid (gs_init_gaussians)."""

    def __init__(self, cam, device="cuda"):
        L.load()
        self.cam = L.make_cameras([cam])[0]
        self.W, self.H = int(cam.width), int(cam.height)
        self.device = torch.device(device)
        self.depth_map = torch.empty(self.W * self.H, dtype=torch.float32, device=self.device)
        self.tracked = torch.empty(self.W * self.H, dtype=torch.uint8, device=self.device)
        self.ws_bytes = L.gs_init_gaussians_workspace_size(self.cam)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.d_count = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.tris = None

    def triangulate(self, xy) -> np.ndarray:
        self.tris = L.gs_delaunay(np.asarray(xy))
        return self.tris

    def densify(self, xy, depth, image: torch.Tensor, tau: float = 0.02, tris: Optional[np.ndarray] = None):
        """Depth map of the keyframe ([H W] on the device; 0 where none)."""
        xy = np.ascontiguousarray(xy, np.int32)
        tris = self.triangulate(xy) if tris is None else np.ascontiguousarray(tris, np.int32)
        self.d_xy = torch.as_tensor(xy, device=self.device)
        self.d_depth = torch.as_tensor(np.ascontiguousarray(depth, np.float32), device=self.device)
        self.d_tris = torch.as_tensor(tris, device=self.device)
        L.gs_densify_depth(self.cam, _p(self.d_xy), _p(self.d_depth), int(xy.shape[0]), _p(self.d_tris),
                           int(tris.shape[0]), _p(image), float(tau), _p(self.depth_map), _p(self.tracked), _stream())
        return self.depth_map

    def fill(self, image: torch.Tensor, tau: float = 0.02):
        """gs_densify_depth again on the points and triangles of the last densify() (no host work)."""
        L.gs_densify_depth(self.cam, _p(self.d_xy), _p(self.d_depth), int(self.d_xy.shape[0]), _p(self.d_tris),
                           int(self.d_tris.shape[0]), _p(image), float(tau), _p(self.depth_map), _p(self.tracked),
                           _stream())

    def init_into(self, image: torch.Tensor, stride: int, out: GaussianParams):
        """gs_init_gaussians_count then gs_init_gaussians into `out` (sized by an earlier count())."""
        L.gs_init_gaussians_count(self.cam, _p(self.depth_map), _p(self.tracked), int(stride), _p(self.d_count),
                                  self.ws.data_ptr(), self.ws_bytes, _stream())
        L.gs_init_gaussians(self.cam, _p(self.depth_map), _p(self.tracked), _p(image), int(stride), out.sh_degree,
                            out.n, out.c_grads(), self.ws.data_ptr(), self.ws_bytes, _stream())

    def count(self, stride: int) -> int:
        L.gs_init_gaussians_count(self.cam, _p(self.depth_map), _p(self.tracked), int(stride), _p(self.d_count),
                                  self.ws.data_ptr(), self.ws_bytes, _stream())
        return int(self.d_count.item())

    def init(self, image: torch.Tensor, stride: int, sh_degree: int, n_out: Optional[int] = None) -> GaussianParams:
        """The new Gaussians of the current depth map (count() first, or pass its result as n_out)."""
        n = self.count(stride) if n_out is None else int(n_out)
        out = GaussianParams.empty(n, sh_degree, self.device)
        L.gs_init_gaussians(self.cam, _p(self.depth_map), _p(self.tracked), _p(image), int(stride), int(sh_degree), n,
                            out.c_grads(), self.ws.data_ptr(), self.ws_bytes, _stream())
        return out


class MappingLoop:
    """The mapping iterations of Sec. III-B over a keyframe window: coarse-to-fine over the Gaussian
    pyramid of the targets, each keyframe on its own schedule (a keyframe added later starts at the
    coarsest level while the others train at full resolution, in one batch of mixed view sizes),
    the loss of eq. (2) (ssim_lambda > 0 adds its SSIM term), Adam, and every `densify_every`
    iterations (1000 in Sec. IV-A) the adaptive density control, after which the iterations
    continue on the new set with the optimiser state handed over.  add_keyframe() initialises the
    new keyframe's Gaussians from its tracked pixels (Sec. III-A) and appends them (zero moments).
    Every step of the method runs in libgs kernels; the loop sequences them, and appending
    Gaussians is a device copy."""

    def __init__(self, params: GaussianParams, cameras, targets, lrs=None, levels: int = 2, schedule=None,
                 ssim_lambda: float = 0.2, densify_every: int = 1000, tile_size: int = 16, graphs: bool = True,
                 generator: Optional[torch.Generator] = None, check_every: int = 100, spatial_order: bool = True,
                 autotune: bool = False, **density_cfg):
        """check_every: iterations between host checks of the pair-capacity overflow flag (also checked
        before every density step); an overflow raises CapacityOverflow.  spatial_order: the set a
        density step makes is put in Morton order of its means (spatially_ordered) before the
        iterations continue; its statistics restart at zero, so only the parameters and moments move.
        autotune: every per-view level batch is autotuned (PyramidMappingStep), again after each
        density step since the set, and with it the best setting, has changed."""
        self.cameras, self.lrs, self.levels = list(cameras), lrs, int(levels)
        self.targets = [t if isinstance(t, torch.Tensor) else pack_images([t], params.means.device)
                        for t in targets]
        self.densify_every = int(densify_every)
        self.check_every = max(1, int(check_every))
        self.generator = generator
        self.spatial_order = bool(spatial_order)
        self.last_order = None  # the permutation of the last reorder (int32, new row k <- row order[k])
        self.density = DensityControl(params.n, cameras, device=params.means.device, **density_cfg)
        self._opts = dict(schedule=schedule, lrs=lrs, graphs=graphs, ssim_lambda=ssim_lambda, tile_size=tile_size,
                          density=self.density, autotune=autotune)
        self.steps = PyramidMappingStep(params, self.cameras, torch.cat(self.targets), levels=self.levels,
                                        **self._opts)
        self.kf_iters = [0] * len(self.cameras)  # iterations each keyframe has trained
        self.iteration = 0
        self.history = []  # (iteration, n) after each density step

    @property
    def params(self) -> GaussianParams:
        return self.steps.params

    def _rebuild(self, params: GaussianParams, adam: FusedAdam, rebuild_pyramid: bool = False):
        pyr = None if rebuild_pyramid else self.steps.pyramid
        self.steps = PyramidMappingStep(params, self.cameras, torch.cat(self.targets), levels=self.levels,
                                        adam=adam, pyramid=pyr, **self._opts)

    def run(self, iterations: int) -> MappingStep:
        st = None
        for _ in range(int(iterations)):
            st = self.steps.run_levels([self.steps.level_at(k) for k in self.kf_iters])
            self.kf_iters = [k + 1 for k in self.kf_iters]
            self.iteration += 1
            densify = self.densify_every > 0 and self.iteration % self.densify_every == 0
            if densify or self.iteration % self.check_every == 0:
                self.steps.check_overflow()
            if densify:
                new_p, new_adam = self.density.apply(self.steps.params, self.steps.adam, generator=self.generator)
                if self.spatial_order and new_p.n > 0:
                    new_p, new_adam, self.last_order = spatially_ordered(new_p, new_adam)
                self._rebuild(new_p, new_adam)
                self.history.append((self.iteration, new_p.n))
        return st

    def add_keyframe(self, cam, target, xy, depth, stride: int = 4, tau: float = 0.02) -> int:
        """Appends keyframe `cam` with its image `target` ([3, H, W]) and the Gaussians initialised
        from its tracked pixels (integer xy, depth); returns how many were added."""
        dev = self.params.means.device
        image = target if isinstance(target, torch.Tensor) else pack_images([target], dev)
        pc = PointCloudInit(cam, device=dev)
        pc.densify(xy, depth, image, tau=tau)
        new = pc.init(image, stride, self.params.sh_degree)
        old, adam = self.params, self.steps.adam
        cat = lambda a, b: torch.cat([a, b]).contiguous()  # noqa: E731
        params = GaussianParams(*[cat(getattr(old, k), getattr(new, k)) for k in PARAM_NAMES], old.sh_degree)
        zeros = new.zeros_like()
        m = GaussianParams(*[cat(getattr(adam.exp_avg, k), getattr(zeros, k)) for k in PARAM_NAMES], old.sh_degree)
        v = GaussianParams(*[cat(getattr(adam.exp_avg_sq, k), getattr(zeros, k)) for k in PARAM_NAMES],
                           old.sh_degree)
        new_adam = FusedAdam(params, params.zeros_like(), adam.lrs, adam.betas, adam.eps, exp_avg=m, exp_avg_sq=v,
                             d_step=adam.d_step)
        # the statistics of the existing Gaussians carry on; the new ones start at zero
        g, a, c = self.density.grad_accum, self.density.abs_accum, self.density.count
        self.density._alloc(params.n)
        self.density.grad_accum[:old.n].copy_(g)
        self.density.abs_accum[:old.n].copy_(a)
        self.density.count[:old.n].copy_(c)
        self.cameras.append(cam)
        self.targets.append(image)
        self.kf_iters.append(0)
        self._rebuild(params, new_adam, rebuild_pyramid=True)
        return new.n
