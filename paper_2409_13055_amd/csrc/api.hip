// C-ABI plumbing of libgs: status strings, thread-local error detail,
// argument validation, view/camera tables and size queries.
#include <cmath>
#include <cstring>
#include <string>

#include "gs_internal.h"

namespace gs {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

gs_status fail(gs_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

gs_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return GS_OK;
}

static bool finite(float x) { return std::isfinite(x); }

gs_status validate_cams(const gs_camera* cams, int32_t n_views) {
  if (!cams) return fail(GS_ERR_INVALID_VALUE, "cams is NULL");
  if (n_views < 1 || n_views > GS_MAX_VIEWS)
    return fail(GS_ERR_INVALID_VALUE, "n_views must be in [1, " + std::to_string(GS_MAX_VIEWS) + "]");
  int64_t px = 0;
  for (int v = 0; v < n_views; ++v) {
    const gs_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > 32768 || c.height > 32768)
      return fail(GS_ERR_INVALID_VALUE, "camera " + std::to_string(v) + ": width/height out of [1, 32768]");
    if (!(c.fx > 0) || !(c.fy > 0) || !finite(c.fx) || !finite(c.fy) || !finite(c.cx) || !finite(c.cy))
      return fail(GS_ERR_INVALID_VALUE, "camera " + std::to_string(v) + ": bad intrinsics");
    for (int k = 0; k < 9; ++k)
      if (!finite(c.R[k])) return fail(GS_ERR_INVALID_VALUE, "camera " + std::to_string(v) + ": non-finite R");
    for (int k = 0; k < 3; ++k)
      if (!finite(c.t[k])) return fail(GS_ERR_INVALID_VALUE, "camera " + std::to_string(v) + ": non-finite t");
    px += (int64_t)c.width * c.height;
  }
  if (px >= (int64_t(1) << 29)) return fail(GS_ERR_INVALID_VALUE, "total pixel count must be < 2^29");
  return GS_OK;
}

gs_status validate_opts(const gs_options* o) {
  if (!o) return fail(GS_ERR_INVALID_VALUE, "opts is NULL");
  if (o->tile_size != 8 && o->tile_size != 16 && o->tile_size != 32)
    return fail(GS_ERR_UNSUPPORTED, "tile_size must be 8, 16 or 32");
  if (o->checkpoint != 0 && o->checkpoint != 1) return fail(GS_ERR_INVALID_VALUE, "checkpoint must be 0 or 1");
  if (!(o->near_plane > 0) || !finite(o->near_plane)) return fail(GS_ERR_INVALID_VALUE, "near_plane must be > 0");
  if (!(o->eps2d >= 0) || !finite(o->eps2d)) return fail(GS_ERR_INVALID_VALUE, "eps2d must be >= 0");
  if (!(o->alpha_min > 0) || !(o->alpha_max > o->alpha_min) || !(o->alpha_max < 1))
    return fail(GS_ERR_INVALID_VALUE, "need 0 < alpha_min < alpha_max < 1");
  if (!(o->t_min > 0) || !(o->t_min < 1)) return fail(GS_ERR_INVALID_VALUE, "need 0 < t_min < 1");
  if (!(o->radius_sigmas > 0) || !finite(o->radius_sigmas))
    return fail(GS_ERR_INVALID_VALUE, "radius_sigmas must be > 0");
  if (!(o->frustum_guard > 0) || !finite(o->frustum_guard))
    return fail(GS_ERR_INVALID_VALUE, "frustum_guard must be > 0");
  for (int k = 0; k < 3; ++k)
    if (!finite(o->bg[k])) return fail(GS_ERR_INVALID_VALUE, "bg must be finite");
  if ((o->flags & ~GS_OPT_WINDOW_LISTS) != 0) return fail(GS_ERR_INVALID_VALUE, "unknown bits in flags");
  if (o->lds_batch != 1 && o->lds_batch != 2) return fail(GS_ERR_UNSUPPORTED, "lds_batch must be 1 or 2");
  return GS_OK;
}

ViewTable make_view_table(const gs_camera* cams, int32_t n_views, int32_t tile) {
  ViewTable vt;
  std::memset(&vt, 0, sizeof vt);
  vt.n_views = n_views;
  vt.tile = tile;
  int32_t to = 0, po = 0, wo = 0;
  for (int v = 0; v < n_views; ++v) {
    ViewGeom& g = vt.v[v];
    g.W = cams[v].width;
    g.H = cams[v].height;
    g.TX = (g.W + tile - 1) / tile;
    g.TY = (g.H + tile - 1) / tile;
    g.tile_off = to;
    g.pix_off = po;
    g.WX = (g.TX + kWinSide - 1) / kWinSide;
    g.WY = (g.TY + kWinSide - 1) / kWinSide;
    g.win_off = wo;
    to += g.TX * g.TY;
    po += g.W * g.H;
    wo += g.WX * g.WY;
  }
  vt.total_windows = wo;
  vt.total_tiles = to;
  vt.total_pixels = po;
  return vt;
}

CamTable make_cam_table(const gs_camera* cams, int32_t n_views, const gs_options* o) {
  CamTable ct;
  std::memset(&ct, 0, sizeof ct);
  for (int v = 0; v < n_views; ++v) {
    const gs_camera& c = cams[v];
    CamF& f = ct.c[v];
    std::memcpy(f.R, c.R, sizeof f.R);
    std::memcpy(f.t, c.t, sizeof f.t);
    f.fx = c.fx;
    f.fy = c.fy;
    f.cx = c.cx;
    f.cy = c.cy;
    for (int k = 0; k < 3; ++k)
      f.centre[k] = -(c.R[k] * c.t[0] + c.R[3 + k] * c.t[1] + c.R[6 + k] * c.t[2]);
    f.limx = o->frustum_guard * 0.5f * (float)c.width / c.fx;
    f.limy = o->frustum_guard * 0.5f * (float)c.height / c.fy;
    f.W = c.width;
    f.H = c.height;
  }
  return ct;
}

}  // namespace gs

extern "C" {

const char* gs_status_string(gs_status s) {
  switch (s) {
    case GS_OK: return "GS_OK";
    case GS_ERR_INVALID_VALUE: return "GS_ERR_INVALID_VALUE";
    case GS_ERR_UNSUPPORTED: return "GS_ERR_UNSUPPORTED";
    case GS_ERR_CAPACITY: return "GS_ERR_CAPACITY";
    case GS_ERR_HIP: return "GS_ERR_HIP";
  }
  return "GS_UNKNOWN_STATUS";
}

const char* gs_last_error(void) { return gs::g_last_error.c_str(); }

int32_t gs_abi_version(void) { return GS_ABI_VERSION; }

void gs_default_options(gs_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tile_size = 16;
  o->checkpoint = 0;
  o->near_plane = 0.2f;
  o->eps2d = 0.3f;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_min = 1e-4f;
  o->radius_sigmas = 3.0f;
  o->frustum_guard = 1.3f;
  o->lds_batch = 1;
}

gs_status gs_total_tiles(const gs_camera* cams, int32_t n_views, int32_t tile_size, int64_t* out) {
  gs_status s = gs::validate_cams(cams, n_views);
  if (s != GS_OK) return s;
  if (!out) return gs::fail(GS_ERR_INVALID_VALUE, "out is NULL");
  if (tile_size != 8 && tile_size != 16 && tile_size != 32)
    return gs::fail(GS_ERR_UNSUPPORTED, "tile_size must be 8, 16 or 32");
  *out = gs::make_view_table(cams, n_views, tile_size).total_tiles;
  return GS_OK;
}

gs_status gs_total_windows(const gs_camera* cams, int32_t n_views, int32_t tile_size, int64_t* out) {
  gs_status s = gs::validate_cams(cams, n_views);
  if (s != GS_OK) return s;
  if (!out) return gs::fail(GS_ERR_INVALID_VALUE, "out is NULL");
  if (tile_size != 8 && tile_size != 16 && tile_size != 32)
    return gs::fail(GS_ERR_UNSUPPORTED, "tile_size must be 8, 16 or 32");
  *out = gs::make_view_table(cams, n_views, tile_size).total_windows;
  return GS_OK;
}

gs_status gs_total_pixels(const gs_camera* cams, int32_t n_views, int64_t* out) {
  gs_status s = gs::validate_cams(cams, n_views);
  if (s != GS_OK) return s;
  if (!out) return gs::fail(GS_ERR_INVALID_VALUE, "out is NULL");
  *out = gs::make_view_table(cams, n_views, 16).total_pixels;
  return GS_OK;
}

}  // extern "C"
