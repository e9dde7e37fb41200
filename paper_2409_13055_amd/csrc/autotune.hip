// Tile-size autotuner.  The tile of the tile-based rasteriser (Sec. III-B) is
// a free parameter: small tiles list each splat in more tiles (more sort and
// staging work), large ones evaluate more entries per pixel.  Which one is
// fastest depends on the splats' footprints and on the views, so the
// candidates are timed on the actual problem: one iteration of projection,
// bin/sort, forward with the L1 term, raster backward and projection
// backward, through the library's own entry points.  The LDS batch of the
// raster kernels (one or two splat records per lane) is timed with each tile
// size on the same buffers.
//
// This is the one call that allocates device memory (its own buffers for each
// candidate, freed before it returns) and the one that synchronises: it is not
// part of the captured iteration.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gs_internal.h"

namespace gs {

namespace {

// Device buffers of one candidate, freed on scope exit.
struct DeviceBuffers {
  std::vector<void*> ptrs;
  ~DeviceBuffers() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  hipError_t alloc(void** out, size_t bytes) {
    *out = nullptr;
    const hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) ptrs.push_back(*out);
    return e;
  }
};

static_assert(GS_AUTOTUNE_MAX_CANDIDATES >= 3 * 2 * 2, "three tile sizes x two LDS batches x two bins forms");

std::mutex g_cache_mu;
std::map<std::vector<int64_t>, gs_autotune_result> g_cache;

std::vector<int64_t> cache_key(const gs_params* p, const gs_camera* cams, int32_t n_views, const gs_options* o,
                               int32_t mask) {
  std::vector<int64_t> key;
  key.push_back((int64_t)std::floor(std::log2((double)std::max<int64_t>(p->n, 1))));
  key.push_back(p->sh_degree);
  key.push_back(o->checkpoint);
  key.push_back((int64_t)(o->flags & ~GS_OPT_WINDOW_LISTS));  // the bins form is a candidate
  key.push_back(mask);
  std::vector<int64_t> res;
  for (int v = 0; v < n_views; ++v) res.push_back((int64_t)cams[v].width << 32 | (int64_t)cams[v].height);
  std::sort(res.begin(), res.end());
  key.insert(key.end(), res.begin(), res.end());
  return key;
}

// Times `iters` iterations at one tile size; *ms < 0 when the candidate cannot run (memory, or a pair
// count beyond the 32-bit index space).  Returns an error only for failures that are not about size.
// Times `iters` iterations at one tile size for each LDS batch of `batches` (n_b of them, into ms[b]
// and pairs[b]); the buffers are allocated once for the tile size.
gs_status time_candidate(const gs_params* params, const gs_camera* cams, int32_t n_views, const gs_options* base,
                         int32_t tile, const int32_t* batches, int n_b, const float* target, int32_t iters,
                         hipStream_t st, float* ms_out, int64_t* pairs_out) {
  for (int b = 0; b < n_b; ++b) {
    ms_out[b] = -1.0f;
    pairs_out[b] = -1;
  }
  int64_t* pairs = pairs_out;  // the pair count is the same for every batch
  gs_options o = *base;
  o.tile_size = tile;
  const ViewTable vt = make_view_table(cams, n_views, tile);
  const int64_t n = params->n, VN = n * n_views, S = n_views * ((n + 63) / 64), Px = vt.total_pixels;
  const int K = (params->sh_degree + 1) * (params->sh_degree + 1);
  DeviceBuffers buf;
  void *rec, *tt, *vis, *vcnt, *ranges, *np, *ovf, *rgb, *tfin = nullptr, *ncon = nullptr, *wsf, *lout, *g2;
  void *gm, *gs_, *gq, *go, *gdc, *grest = nullptr, *ids = nullptr, *wss = nullptr, *wr = nullptr, *ni = nullptr;
  const bool win = (o.flags & GS_OPT_WINDOW_LISTS) != 0;
  size_t fwd_bytes = 0;
  gs_status s = gs_render_fwd_workspace_size(cams, n_views, &o, &fwd_bytes);
  if (s != GS_OK) return s;
  hipError_t e = hipSuccess;
  auto A = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = buf.alloc(p, bytes);
  };
  A(&rec, sizeof(float) * GS_REC_FLOATS * VN);
  A(&tt, sizeof(int32_t) * VN);
  A(&vis, sizeof(uint32_t) * 4 * 64 * S);
  A(&vcnt, sizeof(uint32_t) * S);
  A(&ranges, sizeof(uint32_t) * 2 * vt.total_tiles);
  A(&np, sizeof(int64_t));
  A(&ni, sizeof(int64_t));
  A(&ovf, sizeof(int32_t));
  if (win) A(&wr, sizeof(uint32_t) * 2 * (size_t)std::max(vt.total_windows, 1));
  A(&rgb, sizeof(float) * 3 * Px);
  if (!o.checkpoint) {
    A(&tfin, sizeof(float) * Px);
    A(&ncon, sizeof(int32_t) * Px);
  }
  A(&wsf, fwd_bytes);
  A(&lout, sizeof(float) * n_views);
  A(&g2, sizeof(float) * GS_GRAD2D_FLOATS * VN);
  A(&gm, sizeof(float) * 3 * n);
  A(&gs_, sizeof(float) * 3 * n);
  A(&gq, sizeof(float) * 4 * n);
  A(&go, sizeof(float) * n);
  A(&gdc, sizeof(float) * 3 * n);
  if (K > 1) A(&grest, sizeof(float) * 3 * (K - 1) * n);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return GS_OK;  // skipped
  }
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("gs_autotune: hipMalloc: ") + hipGetErrorString(e));
  const gs_projected proj{static_cast<float*>(rec), static_cast<int32_t*>(tt), static_cast<uint32_t*>(vis),
                          static_cast<uint32_t*>(vcnt)};
  gs_bins bins{nullptr, nullptr, static_cast<uint32_t*>(ranges), 0, static_cast<int64_t*>(np),
               static_cast<int32_t*>(ovf), nullptr, static_cast<uint32_t*>(wr), static_cast<int64_t*>(ni)};
  const gs_image img{static_cast<float*>(rgb), static_cast<float*>(tfin), static_cast<int32_t*>(ncon)};
  gs_loss loss{};
  loss.kind = GS_LOSS_L1;
  loss.target = target;
  loss.loss_out = static_cast<float*>(lout);
  const gs_grads grads{static_cast<float*>(gm), static_cast<float*>(gs_), static_cast<float*>(gq),
                       static_cast<float*>(go), static_cast<float*>(gdc), static_cast<float*>(grest)};
  // pair (and window item) count: a sort with capacity 0 reports it
  size_t ws_bytes = 0;
  if ((s = gs_bin_sort_workspace_size(n, cams, n_views, &o, 0, &ws_bytes)) != GS_OK) return s;
  A(&wss, ws_bytes);
  A(&ids, sizeof(uint32_t) * 2);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return GS_OK;
  }
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("gs_autotune: hipMalloc: ") + hipGetErrorString(e));
  bins.ids = static_cast<uint32_t*>(ids);
  bins.items = static_cast<uint32_t*>(ids);
  if ((s = gs_project(params, cams, n_views, &o, &proj, st)) != GS_OK) return s;
  if ((s = gs_bin_sort(&proj, n, cams, n_views, &o, &bins, wss, ws_bytes, st)) != GS_OK) return s;
  int64_t m = 0, items = 0;
  e = hipMemcpyAsync(&m, np, sizeof m, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&items, ni, sizeof items, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("gs_autotune: ") + hipGetErrorString(e));
  *pairs = m;
  // the capacity bounds the incidences (tile lists) or the window items (window lists)
  const int64_t cap = (int64_t)std::ceil((double)(win ? items : m) * 1.25) + 1024;
  if (cap >= (int64_t(1) << 32) - 1) return GS_OK;  // beyond the 32-bit pair index space: skipped
  if ((s = gs_bin_sort_workspace_size(n, cams, n_views, &o, cap, &ws_bytes)) != GS_OK) return s;
  A(&wss, ws_bytes);
  A(&ids, (win ? sizeof(uint2) : sizeof(uint32_t)) * (size_t)cap);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return GS_OK;
  }
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("gs_autotune: hipMalloc: ") + hipGetErrorString(e));
  bins.ids = win ? nullptr : static_cast<uint32_t*>(ids);
  bins.items = win ? static_cast<uint32_t*>(ids) : nullptr;
  bins.capacity = cap;
  auto iteration = [&]() -> gs_status {
    gs_status r;
    if ((r = gs_project(params, cams, n_views, &o, &proj, st)) != GS_OK) return r;
    if ((r = gs_bin_sort(&proj, n, cams, n_views, &o, &bins, wss, ws_bytes, st)) != GS_OK) return r;
    if ((r = gs_render_fwd(&proj, n, &bins, cams, n_views, &o, &loss, &img, wsf, fwd_bytes, st)) != GS_OK) return r;
    if ((r = gs_raster_bwd(&proj, n, &bins, &img, cams, n_views, &o, &loss, static_cast<float*>(g2), st)) != GS_OK)
      return r;
    return gs_project_bwd(params, &proj, cams, n_views, &o, static_cast<float*>(g2), &grads, st);
  };
  for (int bi = 0; bi < n_b; ++bi) {
    o.lds_batch = batches[bi];
    pairs_out[bi] = *pairs;
    if ((s = iteration()) != GS_OK) return s;  // warm-up
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int it = 0; e == hipSuccess && s == GS_OK && it < iters; ++it) s = iteration();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float total = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&total, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s != GS_OK) return s;
    if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("gs_autotune: events: ") + hipGetErrorString(e));
    int32_t over = 0;
    e = hipMemcpy(&over, ovf, sizeof over, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("gs_autotune: ") + hipGetErrorString(e));
    if (over) return fail(GS_ERR_CAPACITY, "gs_autotune: the pair count grew past its capacity while timing");
    ms_out[bi] = total / (float)iters;
  }
  return GS_OK;
}

}  // namespace

}  // namespace gs

extern "C" gs_status gs_autotune(const gs_params* params, const gs_camera* cams, int32_t n_views,
                                 const gs_options* opts, const float* target, int32_t iters, int32_t candidate_mask,
                                 int32_t refresh, gs_autotune_result* out, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if ((s = validate_params(params)) != GS_OK) return s;
  if (!target) return fail(GS_ERR_INVALID_VALUE, "gs_autotune times the L1 iteration: target is required");
  if (!out) return fail(GS_ERR_INVALID_VALUE, "out is NULL");
  if (iters < 1 || iters > 1000) return fail(GS_ERR_INVALID_VALUE, "iters must be in [1, 1000]");
  if (candidate_mask < 0 || candidate_mask > 127)
    return fail(GS_ERR_INVALID_VALUE,
                "candidate_mask uses bits 0-2 (tiles 8, 16, 32), 3-4 (LDS batch 1, 2) and 5-6 (tile, window lists)");
  const int32_t tmask = (candidate_mask & 7) == 0 ? 7 : (candidate_mask & 7);
  const int32_t bmask = ((candidate_mask >> 3) & 3) == 0 ? 3 : ((candidate_mask >> 3) & 3);
  const int32_t lmask = ((candidate_mask >> 5) & 3) == 0 ? 3 : ((candidate_mask >> 5) & 3);
  const int32_t mask = tmask | (bmask << 3) | (lmask << 5);
  if ((int64_t)n_views * params->n >= (int64_t(1) << 32) - 1) return fail(GS_ERR_INVALID_VALUE, "bad n");
  const std::vector<int64_t> key = cache_key(params, cams, n_views, opts, mask);
  if (!refresh) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *out = it->second;
      out->from_cache = 1;
      return GS_OK;
    }
  }
  hipStream_t st = as_stream(stream);
  gs_autotune_result r{};
  r.tile_size = 0;
  const int32_t tiles[3] = {8, 16, 32};
  int32_t batches[2];
  int n_b = 0;
  for (int b = 0; b < 2; ++b)
    if ((bmask >> b) & 1) batches[n_b++] = b + 1;
  float best = 0.0f;
  for (int k = 0; k < 3; ++k) {
    if (!((tmask >> k) & 1)) continue;
    for (int f = 0; f < 2; ++f) {
      if (!((lmask >> f) & 1)) continue;
      gs_options of = *opts;
      of.flags = f ? (of.flags | GS_OPT_WINDOW_LISTS) : (of.flags & ~GS_OPT_WINDOW_LISTS);
      const int c = r.n_candidates;
      r.n_candidates += n_b;
      for (int b = 0; b < n_b; ++b) {
        r.cand_tile[c + b] = tiles[k];
        r.cand_batch[c + b] = batches[b];
        r.cand_window[c + b] = f;
      }
      if ((s = time_candidate(params, cams, n_views, &of, tiles[k], batches, n_b, target, iters, st, &r.ms[c],
                              &r.pairs[c])) != GS_OK)
        return s;
      for (int b = 0; b < n_b; ++b) {
        if (r.ms[c + b] > 0.0f && (r.tile_size == 0 || r.ms[c + b] < best)) {
          best = r.ms[c + b];
          r.tile_size = tiles[k];
          r.lds_batch = batches[b];
          r.window_lists = f;
        }
      }
    }
  }
  if (r.tile_size == 0) return fail(GS_ERR_CAPACITY, "gs_autotune: no candidate tile size fits in device memory");
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache[key] = r;
  }
  *out = r;
  out->from_cache = 0;
  return GS_OK;
}
