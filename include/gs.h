/*
 * gs.h -- C ABI of the tile-based differentiable 3D Gaussian splatting
 * rasteriser and its optimiser step: the data-parallel hot path of the
 * dense-reconstruction (mapping) module of MGSO (Sec. III-B).
 *
 * The mapping module renders keyframe images of a 3D Gaussian map (each
 * Gaussian carries a position, an orientation quaternion, per-axis scales,
 * an opacity and a colour) with the tile-based differentiable rasteriser of
 * Sec. III-B, whose three stages (Sec. II) are a perspective projection of
 * every Gaussian to a 2D splat, an ordering of the splats of each screen tile
 * by depth, and front-to-back alpha compositing of each pixel.  It optimises
 * the Gaussian parameters by gradient descent on a photometric loss against
 * the captured keyframe images (eq. (2)) with the default 3DGS optimiser
 * configuration (Sec. IV-A).  Several keyframes of
 * the SLAM window (eight by default, Sec. III-A) can be rendered in one call.
 *
 * Conventions shared by every call
 *  - Every pointer inside the structs below is a DEVICE pointer unless
 *    stated otherwise.  The caller allocates and owns all device memory,
 *    workspaces included; the library never allocates, frees or retains it
 *    (gs_render_fwd_noalloc's static per-GPU scratch and gs_autotune's own
 *    temporary buffers aside).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Hot-path calls
 *    only enqueue kernels on it and return; none synchronises, so they may be
 *    captured into a HIP graph.  No call issues hipMemset: buffers that must
 *    start at zero are cleared by the library's own fill kernels.
 *  - Arguments are validated before anything is enqueued; on failure the
 *    call returns GS_ERR_INVALID_VALUE (or GS_ERR_UNSUPPORTED) and leaves the
 *    stream untouched.  A failed kernel launch returns GS_ERR_HIP.  The
 *    detail of the last failure on the calling thread is in gs_last_error().
 *  - Views: up to GS_MAX_VIEWS cameras per call, passed as a HOST array.
 *    View v owns the global tiles [tile_off(v), tile_off(v) + TX_v*TY_v) with
 *    TX_v = ceil(W_v/B), TY_v = ceil(H_v/B), tile_off(v) = sum_{u<v} TX_u*TY_u,
 *    local tile (tx,ty) -> tile_off(v) + ty*TX_v + tx, and the pixels
 *    [pix_off(v), pix_off(v) + H_v*W_v), pix_off(v) = sum_{u<v} H_u*W_u.
 *  - (view, Gaussian) pairs are indexed v*N + i.
 */
#ifndef GS_H_
#define GS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 4
#define GS_MAX_VIEWS 32
#define GS_MAX_SH_DEGREE 3
/* floats per projected record, see gs_projected */
#define GS_REC_FLOATS 12
/* floats per image-space gradient row, see gs_render_bwd */
#define GS_GRAD2D_FLOATS 9
#define GS_MAX_ADAM_GROUPS 8

typedef enum gs_status {
  GS_OK = 0,
  GS_ERR_INVALID_VALUE = 1, /* bad pointer, size or option; nothing enqueued */
  GS_ERR_UNSUPPORTED = 2,   /* valid but not implemented (e.g. tile size 12) */
  GS_ERR_CAPACITY = 3,      /* a caller buffer is too small (host-detectable) */
  GS_ERR_HIP = 4            /* a HIP runtime call failed */
} gs_status;

const char* gs_status_string(gs_status s);
/* Detail of the last failure on the calling thread ("" if none). */
const char* gs_last_error(void);
int32_t gs_abi_version(void);

/* Pinhole keyframe camera (Sec. III-A keyframe poses).  R (row-major) and t
 * map world to camera coordinates, p_c = R p_w + t, with x right, y down and
 * z forward.  Pixel (i, j) is sampled at the point (i, j) of index
 * coordinates, so a camera-frame point projects to
 * (fx x/z + cx - 1/2, fy y/z + cy - 1/2). */
typedef struct gs_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} gs_camera;

/* Gaussian set G of Sec. III-B in optimiser (raw) space, FP32, one row per
 * Gaussian:
 *   means          [n,3]     location
 *   log_scales     [n,3]     scale = exp(log_scales)
 *   quats          [n,4]     rotation, (w,x,y,z), normalised on use; an all-zero
 *                            quaternion culls the Gaussian
 *   opacity_logits [n]       opacity = sigmoid(logit)
 *   sh_dc          [n,3]     colour, constant spherical-harmonic coefficient
 *   sh_rest        [n,K-1,3] higher SH bands, K = (sh_degree+1)^2 (NULL when
 *                            sh_degree == 0)
 * Colour = max(0, sum_k sh_k Y_k(d) + 1/2) per channel, d the unit direction
 * from the camera centre to the mean; sh_degree 0 is the plain-RGB colour the
 * paper adopts (Sec. III-B). */
typedef struct gs_params {
  int64_t n;
  int32_t sh_degree; /* 0..3 */
  int32_t reserved;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh_dc;
  const float* sh_rest;
} gs_params;

/* Constants of the rasteriser.  The paper defers them to the original 3DGS
 * rasteriser (Sec. III-B); gs_default_options() fills the conventional
 * values noted on the right. */
typedef struct gs_options {
  int32_t tile_size;     /* B: 8, 16 or 32 (16) */
  int32_t checkpoint;    /* 1: forward does not store t_final/n_contrib
                            (the backward never needs them) (0) */
  float near_plane;      /* cull when camera depth <= near_plane (0.2) */
  float eps2d;           /* added to the 2D covariance diagonal, px^2 (0.3) */
  float alpha_min;       /* blend only alpha >= alpha_min (1/255) */
  float alpha_max;       /* alpha = min(alpha_max, o*G) (0.99) */
  float t_min;           /* a Gaussian that would take T below t_min ends
                            the pixel and is not blended (1e-4) */
  float radius_sigmas;   /* radius = ceil(radius_sigmas*sqrt(lambda_max)) (3) */
  float frustum_guard;   /* Jacobian uses x/z clamped to +-guard*(W/2)/fx (1.3) */
  float bg[3];           /* background colour (0,0,0) */
  uint32_t flags;        /* GS_OPT_* bits below; other bits must be 0 (0) */
  int32_t lds_batch;     /* splat records each lane of a raster workgroup
                            stages into LDS per batch: 1 or 2 (1); the
                            batch is lds_batch x the workgroup's threads.
                            Every output is the same for either value. */
} gs_options;

/* gs_options.flags: the bins are window lists (see gs_bins) instead of tile
 * lists.  gs_bin_sort then stops after the window lists, and every raster
 * call takes each tile's entries from its window's list. */
#define GS_OPT_WINDOW_LISTS 1u

void gs_default_options(gs_options* opts);

/* Projected (view, Gaussian) records, FP32, [n_views*n][GS_REC_FLOATS]:
 *   0 mean_x  1 mean_y  2 conic_a  3 conic_b  4 conic_c  5 opacity
 *   6 r  7 g  8 b  9 depth  10 extents (int32 bits)  11 flags (uint32 bits)
 * conic (a,b,c) is the inverse of the dilated 2D covariance S = [[A,B],[B,C]].
 * extents = rx | ry << 16, the half-extents in pixels of the pair's tile
 * rect: with r = ceil(radius_sigmas sqrt(lambda_max(S))) and
 * thr = 2 ln(opacity / (alpha_min (1 - 1e-3))), rx = min(r, ceil(sqrt(thr A)) + 1),
 * ry = min(r, ceil(sqrt(thr C)) + 1), all at most 32767: the box where the
 * Gaussian can still reach alpha_min, inside the radius_sigmas square, so the
 * rect renders like the full square.  The tile rect is
 * [floor((mean_x - rx)/B), floor((mean_x + rx + B - 1)/B)) (FP32, clamped to
 * the grid), likewise in y.  extents 0 marks a culled pair (behind the near
 * plane, degenerate, opacity <= alpha_min (1 - 1e-3), or no tile touched).
 * flags bits 0-2: colour channel clamped at 0; bits 3-4: frustum guard active
 * in x / y.  tiles_touched [n_views*n] = tile count of the pair's rect (0 when
 * culled).  gs_project writes the record of a visible pair (tiles_touched > 0)
 * only: the row of a culled pair keeps whatever it held, and no call reads it
 * (every later stage reaches records through the tile lists).
 * vis, vis_count: the visible pairs (tiles_touched > 0) compacted by blocks of
 * 64 Gaussians, the hand-off from gs_project to gs_bin_sort.  With
 * S = ceil(n/64) segments per view, segment s = v*S + b holds the visible
 * pairs of view v among Gaussians [64 b, 64 b + 64) in ascending i:
 * vis_count [n_views*S] holds their number and vis [n_views*S*64][4] (uint32,
 * 16-byte aligned) holds at slots [64 s, 64 s + vis_count[s]) one entry each:
 * x0 | x1 << 16, y0 | y1 << 16 (the tile rect [x0,x1) x [y0,y1) in the view's
 * grid, as documented at gs_bin_sort), v*n+i, and the FP32 bits of the depth.
 * Slots past a segment's count are not written. */
typedef struct gs_projected {
  float* rec;
  int32_t* tiles_touched;
  uint32_t* vis;
  uint32_t* vis_count;
} gs_projected;

/* Bins, in one of two forms chosen by GS_OPT_WINDOW_LISTS.
 *
 * Tile lists (the flag clear).  keys [capacity] (may be NULL: not written),
 * ids [capacity], ranges [total_tiles][2].  After gs_bin_sort the first M
 * entries of ids hold v*N+i of every (pair, tile) incidence ordered by
 * (global tile, FP32 bit pattern of the depth, v*N+i); keys[p] =
 * (tile << 32) | depth bits; ranges[t] = [first, last+1) of tile t, (0,0) for
 * an empty tile.  d_overflow receives 1 when M > capacity.
 *
 * Window lists (the flag set).  A binning window is a block of 8 x 8 tiles of
 * one view: window (wx, wy) of view v has global index win_off(v) +
 * wy * WX(v) + wx, WX(v) = ceil(TX(v) / 8), windows numbered view by view
 * (gs_total_windows gives their count W).  items [capacity][2] (8-byte
 * aligned) holds, window after window, one item per (pair, window) whose
 * tile rect meets the window: (v*N+i, lx0 | lx1 << 4 | ly0 << 8 | ly1 << 12),
 * the rect clipped to the window in the window's tile coordinates,
 * [lx0, lx1) x [ly0, ly1) inside [0, 8]^2.  Within a window the items are
 * ordered by (FP32 bit pattern of the depth, v*N+i).  win_ranges [2][W]:
 * win_ranges[w] = first item of window w, win_ranges[W + w] = one past its
 * last ((0, 0) for an empty window).  The tile list of tile (tx, ty) is then
 * the items of its window (tx / 8, ty / 8) whose clipped rect covers
 * (tx mod 8, ty mod 8), in window order: the same entries in the same order
 * as the tile-list form.  d_num_items (device int64, may be NULL) receives
 * the item count E; d_overflow receives 1 when E > capacity.  ids, keys and
 * ranges are not used.
 *
 * Both forms: d_num_pairs (device int64) receives M, the number of
 * (pair, tile) incidences.  On overflow the lists are undefined, every range
 * is empty (a raster call then renders the background), and the caller must
 * grow the buffers and call again (d_overflow 0 otherwise). */
typedef struct gs_bins {
  uint64_t* keys;
  uint32_t* ids;
  uint32_t* ranges;
  int64_t capacity;
  int64_t* d_num_pairs;
  int32_t* d_overflow;
  uint32_t* items;
  uint32_t* win_ranges;
  int64_t* d_num_items;
} gs_bins;

/* Rendered views.  rgb [sum_v 3*H_v*W_v]: view v at 3*pix_off(v), planar
 * [3][H_v][W_v]; t_final (final transmittance) and n_contrib (1 + list
 * position of the last blended Gaussian, 0 if none) [sum_v H_v*W_v]; both
 * may be NULL when options.checkpoint is set.  The backward reads only rgb. */
typedef struct gs_image {
  float* rgb;
  float* t_final;
  int32_t* n_contrib;
} gs_image;

typedef enum gs_loss_kind {
  GS_LOSS_NONE = 0,
  GS_LOSS_L1 = 1,       /* L1 term of eq. (2) against `target` */
  GS_LOSS_EXTERNAL = 2  /* the caller supplies dL/dimage in `dl_dimage` */
} gs_loss_kind;

/* Photometric loss.  L1: L = sum_v mean_{c,y,x} |I_r - I_gt| (the L1 term of
 * eq. (2) summed over the rendered views), dL/dI_r = sign(I_r - I_gt) /
 * (3 H_v W_v) with sign(0) = 0.  target and dl_dimage use the rgb layout of
 * gs_image.  loss_out (device, [n_views], may be NULL): gs_render_fwd writes
 * each view's L1 term there. */
typedef struct gs_loss {
  int32_t kind;
  int32_t reserved;
  const float* target;
  const float* dl_dimage;
  float* loss_out;
} gs_loss;

/* Gradients of the raw parameters, same shapes as gs_params; gs_render_bwd
 * ADDS into them (the caller clears them once per iteration), so per-view
 * calls and one batched call both sum over views. */
typedef struct gs_grads {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh_dc;
  float* sh_rest;
} gs_grads;

/* ---------------------------------------------------------------- queries */
/* Total tiles / pixels of a set of views at a tile size (host only). */
gs_status gs_total_tiles(const gs_camera* cams, int32_t n_views, int32_t tile_size, int64_t* out);
gs_status gs_total_pixels(const gs_camera* cams, int32_t n_views, int64_t* out);
/* Binning windows (8 x 8 tiles of one view) of a set of views at a tile size. */
gs_status gs_total_windows(const gs_camera* cams, int32_t n_views, int32_t tile_size, int64_t* out);
/* Workspace bytes of gs_bin_sort for n Gaussians, these views and the
 * capacity of the bins (gs_bins.capacity: incidences for tile lists, items
 * for window lists). */
gs_status gs_bin_sort_workspace_size(int64_t n, const gs_camera* cams, int32_t n_views, const gs_options* opts,
                                     int64_t pair_capacity, size_t* bytes);
/* Workspace bytes of gs_render_fwd (per-tile loss partials) and
 * gs_render_bwd (the [n_views*n][9] image-space gradient buffer). */
gs_status gs_render_fwd_workspace_size(const gs_camera* cams, int32_t n_views, const gs_options* opts,
                                       size_t* bytes);
gs_status gs_render_bwd_workspace_size(int64_t n, int32_t n_views, size_t* bytes);

/* --------------------------------------------------------------- hot path */

/* Projection (Sec. II, first stage of the rasteriser; Gaussian
 * parameterisation of Sec. III-B).  For every Gaussian i and view v: camera
 * point t = R mean + t; cull if t_z <= near_plane; image mean; 2D covariance
 * J W Sigma W^T J^T + eps2d I with Sigma = R(q) S S^T R(q)^T (local affine
 * approximation of the perspective map, frustum guard on x/z and y/z);
 * conic; radius; tile rect; colour; opacity; writes out->tiles_touched for
 * all n_views*n pairs, out->rec for the visible ones (tiles_touched > 0), and
 * the visible pairs' entries to out->vis / out->vis_count.  Parameters are read once for all views. */
gs_status gs_project(const gs_params* params, const gs_camera* cams, int32_t n_views, const gs_options* opts,
                     const gs_projected* out, void* stream);

/* Tile binning and depth sort (Sec. II, second stage; tile-based
 * rasterisation of Sec. III-B).  Every pair with tiles_touched > 0 is
 * assigned to each tile of its rect [floor((m-r)/B), floor((m+r+B-1)/B))
 * (computed in FP32, clamped to the view's grid); the (tile, id) incidences
 * are ordered as documented at gs_bins (a stable LSD radix sort on the
 * 64-bit key, ties broken by ascending v*N+i).  The pairs and their rects are
 * read from proj->vis / proj->vis_count as gs_project wrote them, which must
 * be for the same n, cameras and n_views (their ids number the views of that
 * call; a sub-batch of views is projected by a call of its own); proj->rec is
 * read for the depths of bins->keys.  With GS_OPT_WINDOW_LISTS the call
 * writes the window lists instead (every pair listed once per window its
 * rect meets, then a stable sort on the window index) and no tile list.
 * `workspace` must hold gs_bin_sort_workspace_size() bytes for the same
 * arguments. */
gs_status gs_bin_sort(const gs_projected* proj, int64_t n, const gs_camera* cams, int32_t n_views,
                      const gs_options* opts, const gs_bins* bins, void* workspace, size_t workspace_bytes,
                      void* stream);

/* Forward rasterisation (Sec. II, third stage).  For every
 * pixel, over its tile's list in order: power = -(a dx^2 + c dy^2)/2 - b dx dy
 * with d = pixel - mean (skip if power > 0), alpha = min(alpha_max,
 * opacity exp(power)) (skip if alpha < alpha_min); stop before a Gaussian
 * that would take T below t_min; C += colour alpha T; T *= 1 - alpha.
 * Output C + T bg.  With loss->kind == GS_LOSS_L1 and loss->loss_out set,
 * also writes the per-view L1 term.  `workspace` must hold
 * gs_render_fwd_workspace_size() bytes (may be NULL when no loss value is
 * requested).  Reads the pair count from bins->d_num_pairs. */
gs_status gs_render_fwd(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_camera* cams,
                        int32_t n_views, const gs_options* opts, const gs_loss* loss, const gs_image* out,
                        void* workspace, size_t workspace_bytes, void* stream);

/* gs_render_fwd without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as gs_render_fwd;
 * the per-tile L1 partial sums live in a static array of the library, one per
 * GPU, held until the process ends (GS_NOALLOC_MAX_TILES floats, 4 MiB).  A
 * call that requests the loss value with more than GS_NOALLOC_MAX_TILES tiles
 * returns GS_ERR_CAPACITY and enqueues nothing.  No call allocates or frees
 * memory; its first call on a device looks up that device's array.  Calls
 * that overlap on one GPU (other streams, other threads) share the array and
 * race: serialise them.  Every tile's partial sum is written before it is
 * read, so nothing needs clearing between calls. */
#define GS_NOALLOC_MAX_TILES (1 << 20)
gs_status gs_render_fwd_noalloc(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_camera* cams,
                                int32_t n_views, const gs_options* opts, const gs_loss* loss, const gs_image* out,
                                void* stream);

/* Backward of the rasteriser and the projection (the differentiable part of
 * Sec. III-B): dL/dimage from `loss` (L1 of eq. (2), or external), then for
 * every pixel one front-to-back sweep over its list with the forward's
 * decisions, giving d/d(mean2d, conic, opacity, colour) of each blended
 * Gaussian (the colour behind entry k is the rendered value img->rgb minus
 * the colour blended up to k, so t_final and n_contrib are not read), summed
 * per (view, Gaussian) into the image-space gradient buffer held in
 * `workspace` ([n_views*n][9] floats, order mean_x, mean_y, conic a, b, c,
 * opacity, r, g, b; readable by the caller after the call), then chained
 * through the projection to the raw parameters and added into `grads`.
 * img->rgb must be the image gs_render_fwd wrote for these inputs.
 * `workspace` must hold gs_render_bwd_workspace_size() bytes. */
gs_status gs_render_bwd(const gs_params* params, const gs_projected* proj, const gs_bins* bins,
                        const gs_image* img, const gs_camera* cams, int32_t n_views, const gs_options* opts,
                        const gs_loss* loss, const gs_grads* grads, void* workspace, size_t workspace_bytes,
                        void* stream);

/* The two stages of gs_render_bwd, for callers that hold image-space
 * gradients of their own or time the stages separately.
 *
 * gs_raster_bwd: backward of the blending only (Sec. II / III-B): ADDS, for
 * every (view, Gaussian) pair, d(loss)/d(mean_x, mean_y, conic a, b, c,
 * opacity, r, g, b) into grad2d ([n_views*n][9] FP32, device; the caller
 * clears it).  Loss and image semantics as gs_render_bwd.
 *
 * gs_project_bwd: backward of the projection: chains grad2d (same layout)
 * through gs_project's mapping to the raw parameters and ADDS the result into
 * `grads`, summed over views.  It reads proj->tiles_touched only (pairs with
 * 0 are skipped), which must be what gs_project wrote for these parameters,
 * cameras and options; the rest of the projection is recomputed. */
gs_status gs_raster_bwd(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_image* img,
                        const gs_camera* cams, int32_t n_views, const gs_options* opts, const gs_loss* loss,
                        float* grad2d, void* stream);
gs_status gs_project_bwd(const gs_params* params, const gs_projected* proj, const gs_camera* cams, int32_t n_views,
                         const gs_options* opts, const float* grad2d, const gs_grads* grads, void* stream);

/* Work counts of the blending as defined per pixel (Sec. II), for roofline
 * accounting: d_counts (device int64[3], overwritten) receives, summed over
 * all pixels of all views, [0] the list entries whose alpha is evaluated
 * until the pixel stops (its list end, or the entry that would take T below
 * t_min, inclusive), [1] the (pixel, Gaussian) pairs blended, [2] the
 * contributor counts n_contrib.  Reads the same inputs as gs_render_fwd and
 * writes nothing else. */
gs_status gs_render_stats(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_camera* cams,
                          int32_t n_views, const gs_options* opts, int64_t* d_counts, void* stream);

/* One Adam step over up to GS_MAX_ADAM_GROUPS parameter groups in a single
 * launch (gradient descent of Sec. III-B with the default 3DGS optimiser of
 * Sec. IV-A): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), every element
 * (no visibility mask), t = *d_step + 1.  d_step (device int32) is then
 * incremented, so graph replays need no host scalars.  With zero_grad != 0
 * the gradient is cleared after use.  Every pointer of a group is a device
 * pointer to numel FP32 values. */
typedef struct gs_adam_group {
  float* param;
  float* grad;
  float* exp_avg;
  float* exp_avg_sq;
  int64_t numel;
  float lr;
  int32_t reserved;
} gs_adam_group;

gs_status gs_adam_step(const gs_adam_group* groups /* host array */, int32_t n_groups, double beta1, double beta2,
                       double eps, int32_t* d_step, int32_t zero_grad, void* stream);

/* Projection backward fused with the Adam step (the backward of Sec. III-B
 * followed by the optimiser step of Sec. IV-A, without the raw-parameter
 * gradients going through memory): for every Gaussian the gradient is formed
 * as by gs_project_bwd from grad2d (summed over views; 0 for a Gaussian no
 * view sees) and used at once for one Adam step of each of its parameters as
 * by gs_adam_step (same hyper-parameters, t = *d_step + 1), after which
 * *d_step is incremented.  The result equals gs_project_bwd into zeroed
 * gradients followed by gs_adam_step, bit for bit.  `groups` is a host array
 * of the 6 parameter groups in the order means, log_scales, quats,
 * opacity_logits, sh_dc, sh_rest: group k's param must be the array `params`
 * points to for it (read by the projection, then updated in place; a group
 * with numel 0 may have NULL pointers), numel = n * width (3, 3, 4, 1, 3,
 * 3 ((D+1)^2 - 1)), exp_avg / exp_avg_sq its moments (updated in place); grad
 * is not used.  proj->tiles_touched as for gs_project_bwd. */
gs_status gs_project_bwd_adam(const gs_params* params, const gs_projected* proj, const gs_camera* cams,
                              int32_t n_views, const gs_options* opts, const float* grad2d,
                              const gs_adam_group* groups /* host array [6] */, double beta1, double beta2, double eps,
                              int32_t* d_step, void* stream);

/* Photometric loss with its SSIM term (eq. (2); the L1-only loss is
 * GS_LOSS_L1 inside gs_render_fwd / gs_raster_bwd).  Reading of eq. (2),
 * printed garbled: per view, loss_v = (1 - lambda) L1_v + lambda (1 - SSIM_v),
 * L1_v = mean |I - I_gt| and SSIM_v the mean SSIM map over the view's pixels
 * and 3 channels; SSIM per channel with an 11 x 11 Gaussian window (sigma
 * 1.5, normalised), zero-padded same-size filtering, C1 = 0.01^2,
 * C2 = 0.03^2 (3DGS uses lambda = 0.2).  image, target: [sum_v 3 H_v W_v]
 * FP32, planar per view and packed by view as in gs_image.rgb.  Writes
 * loss_out[v] (may be NULL) and dl_dimage = d(sum_v loss_v)/d image, same
 * layout (may be NULL; not both NULL).  dl_dimage feeds gs_raster_bwd /
 * gs_render_bwd as GS_LOSS_EXTERNAL.  lambda in [0, 1].  `workspace` must
 * hold gs_photometric_loss_workspace_size() bytes (36 bytes per pixel for the
 * gradient's intermediate maps). */
gs_status gs_photometric_loss_workspace_size(const gs_camera* cams, int32_t n_views, size_t* bytes);
gs_status gs_photometric_loss(const gs_camera* cams, int32_t n_views, const float* image, const float* target,
                              float lambda, float* loss_out, float* dl_dimage, void* workspace,
                              size_t workspace_bytes, void* stream);

/* --------------------------------------------------------- memory layout
 * The order of the Gaussians in the parameter arrays is free (every call
 * treats them as a set; only ties between equal depths are broken by the
 * index).  gs_spatial_order gives an order that keeps the Gaussians of each
 * run of 64 consecutive indices close together in space, so the projection
 * and its backward, which walk the Gaussians in wavefronts of 64 and skip the
 * views that see none of a wavefront's Gaussians, skip far more of them (the
 * projection of 2M Gaussians into 16 views: 0.62 -> 0.37 ms): order[k] (device,
 * [n] uint32, written) is the index of the Gaussian that goes to position k,
 * the Gaussians sorted stably by the Morton (Z-order) code of their means,
 * each axis cut into 1024 cells over the means' bounding box (cell =
 * min(1023, floor((m - lo) * (1024 / (hi - lo)))) in FP32; a flat axis and
 * a NaN coordinate give cell 0).  `workspace` must hold
 * gs_spatial_order_workspace_size() bytes.  gs_gather_rows applies such an
 * order to one array of rows: dst[k][c] = src[order[k]][c] for rows of
 * `width` floats (an order entry >= n gives a NaN row; src and dst must not
 * overlap); applied to every parameter array and, during training, to the
 * optimiser's moments, it reorders the Gaussian set. */
gs_status gs_spatial_order_workspace_size(int64_t n, size_t* bytes);
gs_status gs_spatial_order(const float* means, int64_t n, uint32_t* order, void* workspace, size_t workspace_bytes,
                           void* stream);
gs_status gs_gather_rows(const float* src, int64_t n, int32_t width, const uint32_t* order, float* dst,
                         void* stream);

/* ------------------------------------------------------------- autotuning
 * The tile size of the tile-based rasterisation (Sec. III-B), the LDS batch
 * of the raster kernels (gs_options.lds_batch) and the form of the bins
 * (GS_OPT_WINDOW_LISTS) are free parameters: every form gives the same
 * images, and which is fastest depends on the problem (window lists save
 * the sort its tile lists but make a tile scan its window's list, which
 * pays where pixels stop early and costs where tiles walk their whole
 * lists).  gs_autotune picks all three by timing the actual problem: for
 * each candidate (bits 0-2 of candidate_mask: tile 8, 16, 32; bits 3-4: LDS
 * batch 1, 2; bits 5-6: tile lists, window lists; a group with no bit set
 * means all of it) one warm-up and `iters` timed iterations of gs_project,
 * gs_bin_sort, gs_render_fwd with the L1 term against `target` (rgb layout
 * of gs_image, device), gs_raster_bwd and gs_project_bwd on `stream`, at
 * opts with tile_size, lds_batch and the bins flag replaced.  Host-side and
 * synchronising, NOT for graph capture; the only call that allocates device
 * memory (its own buffers per tile size and form, all freed before it
 * returns).  A candidate that does not fit in device memory or whose list
 * count exceeds the 32-bit index space is skipped (ms -1); GS_ERR_CAPACITY
 * when none fits.  Results are cached for the life of the process by
 * (floor(log2 n), the multiset of view resolutions, sh_degree, checkpoint,
 * the other option flags, candidate mask); refresh != 0 times again.  The
 * parameters are not modified. */
#define GS_AUTOTUNE_MAX_CANDIDATES 12
typedef struct gs_autotune_result {
  int32_t tile_size;     /* the fastest candidate's tile size */
  int32_t lds_batch;     /* its LDS batch */
  int32_t window_lists;  /* 1: its bins are window lists (set GS_OPT_WINDOW_LISTS), 0: tile lists */
  int32_t from_cache;    /* 1: taken from the cache, nothing timed */
  int32_t n_candidates;  /* candidates timed, in the order of the arrays */
  int32_t cand_tile[GS_AUTOTUNE_MAX_CANDIDATES];
  int32_t cand_batch[GS_AUTOTUNE_MAX_CANDIDATES];
  int32_t cand_window[GS_AUTOTUNE_MAX_CANDIDATES];
  float ms[GS_AUTOTUNE_MAX_CANDIDATES];      /* mean milliseconds of one iteration at each (-1: skipped) */
  int64_t pairs[GS_AUTOTUNE_MAX_CANDIDATES]; /* (tile, Gaussian) incidences at each (-1: not reached) */
} gs_autotune_result;

gs_status gs_autotune(const gs_params* params, const gs_camera* cams, int32_t n_views, const gs_options* opts,
                      const float* target, int32_t iters, int32_t candidate_mask, int32_t refresh,
                      gs_autotune_result* out, void* stream);

/* ------------------------------------------------- adaptive density control
 * Sec. III-B: every densification interval (1000 iterations, Sec. IV-A)
 * Gaussians with a high homodirectional view-space position gradient (AbsGS)
 * are split when large and cloned when small, with the 3DGS split and clone
 * parameters, and Gaussians of low opacity are pruned.  Readings (the paper
 * gives no formulas):
 *  - gs_raster_bwd_abs: gs_raster_bwd that also ADDS into abs_grad2d
 *    ([n_views*n][2] FP32, device, caller-cleared) the homodirectional
 *    gradient of AbsGS, per (view, Gaussian) pair the sums over pixels of
 *    |dL_p/dmean_x| and |dL_p/dmean_y| (pixel units; dL_p the loss through
 *    pixel p's colour alone); grad2d as for gs_raster_bwd.
 *  - gs_density_accumulate: for every pair with tiles_touched > 0, adds the
 *    Euclidean norm of (W/2 g_x, H/2 g_y) (the gradient in normalised device
 *    units, as in 3DGS) of grad2d's mean part to stats->grad_accum[i], that of
 *    abs_grad2d to stats->abs_accum[i], and 1 to stats->count[i].  proj is the
 *    projection of the iteration that produced the gradients.
 *  - gs_density_plan: classifies every Gaussian (decisions in FP32; the
 *    thresholds are formed in double from cfg and rounded to FP32):
 *    selected = count > 0 and abs_accum >= grad_threshold * count;
 *    pruned = logit < logit(min_opacity); a pruned Gaussian is dropped;
 *    otherwise a selected one with max log-scale > log(percent_dense * extent)
 *    is split (dropped, two children), another selected one is kept and
 *    cloned, an unselected one kept.  Writes d_counts[0..2] (device) = kept,
 *    cloned, split, and the classes into `workspace`
 *    (gs_density_workspace_size(n) bytes), which gs_density_apply reads.
 *  - gs_density_apply: writes the new set of n_out = kept + cloned + 2 split
 *    Gaussians (the caller reads d_counts and allocates): the kept originals,
 *    then the clones (exact copies), then every split's first child, then
 *    every split's second child, each in the original order.  Child k of the
 *    q-th split Gaussian has mean mu + R (s * eps[6 q + 3 k .. +3]) (R the
 *    rotation of the normalised quaternion, s = exp(log_scales), eps standard
 *    normal draws supplied by the caller, n_eps >= 6 * split floats) and
 *    log-scales minus log(split_scale_div); its other parameters are the
 *    parent's.  exp_avg / exp_avg_sq (the Adam moments, same layout as the
 *    parameters) are copied for kept Gaussians and zero for new ones.  Rows at
 *    or past n_out, and children whose eps lie past n_eps, are not written.
 *    The outputs must not overlap the inputs.  The statistics restart at zero
 *    for the new set (the caller clears new arrays).
 *  - gs_scene_extent (host only): 1.1 times the largest distance of a camera
 *    centre from the centres' mean (the 3DGS scene extent).
 *  - gs_default_density_config: the 3DGS values (grad_threshold 0.0002,
 *    percent_dense 0.01, min_opacity 0.005, split_scale_div 1.6), extent 1. */
typedef struct gs_density_config {
  float grad_threshold;
  float percent_dense;
  float min_opacity;
  float split_scale_div;
  float extent;
} gs_density_config;

typedef struct gs_density_stats {
  float* grad_accum; /* [n] */
  float* abs_accum;  /* [n] */
  int32_t* count;    /* [n] */
} gs_density_stats;

gs_status gs_raster_bwd_abs(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_image* img,
                            const gs_camera* cams, int32_t n_views, const gs_options* opts, const gs_loss* loss,
                            float* grad2d, float* abs_grad2d, void* stream);
void gs_default_density_config(gs_density_config* cfg);
gs_status gs_scene_extent(const gs_camera* cams, int32_t n_views, float* extent);
gs_status gs_density_accumulate(const gs_projected* proj, int64_t n, const gs_camera* cams, int32_t n_views,
                                const float* grad2d, const float* abs_grad2d, const gs_density_stats* stats,
                                void* stream);
/* gs_project_bwd_adam followed by gs_density_accumulate of the same grad2d
 * and abs_grad2d, in one pass over grad2d (the statistics are formed in the
 * projection backward's view loop); the results equal the two calls', bit
 * for bit. */
gs_status gs_project_bwd_adam_stats(const gs_params* params, const gs_projected* proj, const gs_camera* cams,
                                    int32_t n_views, const gs_options* opts, const float* grad2d,
                                    const gs_adam_group* groups /* host array [6] */, double beta1, double beta2,
                                    double eps, int32_t* d_step, const float* abs_grad2d,
                                    const gs_density_stats* stats, void* stream);
gs_status gs_density_workspace_size(int64_t n, size_t* bytes);
gs_status gs_density_plan(const gs_params* params, const gs_density_stats* stats, const gs_density_config* cfg,
                          int32_t* d_counts, void* workspace, size_t workspace_bytes, void* stream);
gs_status gs_density_apply(const gs_params* params, const gs_params* exp_avg, const gs_params* exp_avg_sq,
                           const gs_density_config* cfg, const float* eps, int64_t n_eps, int64_t n_out,
                           const gs_grads* out_params, const gs_grads* out_exp_avg, const gs_grads* out_exp_avg_sq,
                           const void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------- point-cloud densification
 * Sec. III-A: the image is triangulated (Delaunay) with the tracked pixels as
 * vertices and the pixels of low-gradient regions take the mean depth of
 * their triangle's vertices; Sec. III-B: new Gaussians start at the points
 * with their colour.  Readings (the paper gives no formulas):
 *  - gs_delaunay (host only): a Delaunay triangulation of the convex hull of
 *    n >= 3 distinct, not all collinear points with integer coordinates in
 *    [0, 32768) (xy host [n][2]), exact (integer predicates; one of the valid
 *    triangulations where four points are cocircular).  Writes *n_tris and,
 *    when max_tris suffices (at most 2 n - 5), tris (host [n_tris][3]) with
 *    every triangle's smallest index first, its orientation kept, the
 *    triangles in lexicographic order; GS_ERR_CAPACITY otherwise.
 *  - gs_densify_depth: depth_map [H W] (device) = 0, then the depth of each
 *    tracked pixel (xy device [n][2], depth device [n], > 0), then for each
 *    triangle (tris device [n_tris][3]) the mean depth of its vertices on the
 *    pixels it owns that are not tracked and of low gradient.  A pixel belongs
 *    to the triangle whose closed interior holds it; an edge shared by two
 *    triangles goes to one: edge a -> b of a positively oriented triangle is
 *    its own when b.y > a.y, or b.y == a.y and b.x < a.x.  Low gradient: grey
 *    = (r + g + b) / 3 of `image` ([3][H][W] FP32, device), central
 *    differences (one-sided at the border), gx^2 + gy^2 < tau^2, each step an
 *    FP32 operation.  tracked [H W] (device bytes) = 1 at tracked pixels.
 *    Points outside the image and triangles with an index outside [0, n) are
 *    skipped.  The camera gives W and H.
 *  - gs_init_gaussians_count, then gs_init_gaussians: one new Gaussian per
 *    pixel with a depth on the grid x % stride == 0, y % stride == 0 (tracked
 *    pixels always), in row-major order; the count goes to d_count (device),
 *    the classes to `workspace` (gs_init_gaussians_workspace_size bytes),
 *    which the second call reads.  Mean: the pixel's index coordinate (x, y)
 *    unprojected at its depth through `cam`; sh_dc = (colour - 1/2) / SH_C0;
 *    quaternion (1, 0, 0, 0); opacity logit log(0.1 / 0.9); log-scales
 *    log(stride * depth / fx) (isotropic: the pixel footprint); sh_rest 0
 *    (sh_degree gives its width).  out holds n_out rows (the count); rows past
 *    n_out are not written. */
gs_status gs_delaunay(const int32_t* xy, int32_t n, int32_t* tris, int32_t max_tris, int32_t* n_tris);
gs_status gs_densify_depth(const gs_camera* cam, const int32_t* xy, const float* depth, int32_t n,
                           const int32_t* tris, int32_t n_tris, const float* image, float tau, float* depth_map,
                           uint8_t* tracked, void* stream);
gs_status gs_init_gaussians_workspace_size(const gs_camera* cam, size_t* bytes);
gs_status gs_init_gaussians_count(const gs_camera* cam, const float* depth_map, const uint8_t* tracked,
                                  int32_t stride, int32_t* d_count, void* workspace, size_t workspace_bytes,
                                  void* stream);
gs_status gs_init_gaussians(const gs_camera* cam, const float* depth_map, const uint8_t* tracked,
                            const float* image, int32_t stride, int32_t sh_degree, int64_t n_out,
                            const gs_grads* out, const void* workspace, size_t workspace_bytes, void* stream);

/* Gaussian pyramid of the ground-truth images for coarse-to-fine training
 * (Sec. III-B, after Photo-SLAM: the images are repeatedly smoothed and
 * down-sampled, and the loss uses coarse levels first).  Reading (the paper
 * gives no filter): one level is the REDUCE step of Burt and Adelson's
 * Gaussian pyramid, the separable binomial window (1, 4, 6, 4, 1) / 16
 * centred on every second pixel, output ceil(W/2) x ceil(H/2), the border
 * reflected without repeating the edge pixel (index -1 reads 1, index W reads
 * W - 2).
 *
 * gs_pyramid_camera (host only, no device work): *out = the camera that
 * samples `levels` reductions of cam's image, each halving fx and fy,
 * mapping cx -> cx / 2 + 1/4 and cy -> cy / 2 + 1/4 (output pixel x' sits at
 * input index 2 x') and width, height -> ceil(/2).  levels in [0, 15]; cam
 * and out are host pointers (may alias).
 *
 * gs_pyramid_reduce: one level for every view.  cams (host array, n_views in
 * [1, GS_MAX_VIEWS]) are the cameras of the src images; src [sum_v 3 H_v W_v]
 * and dst [sum_v 3 ceil(H_v/2) ceil(W_v/2)] are FP32, planar per view and
 * packed by view as gs_image.rgb (dst in the layout of the level cameras).
 * src and dst must not overlap (GS_ERR_INVALID_VALUE). */
gs_status gs_pyramid_camera(const gs_camera* cam, int32_t levels, gs_camera* out);
gs_status gs_pyramid_reduce(const gs_camera* cams, int32_t n_views, const float* src, float* dst, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H_ */
