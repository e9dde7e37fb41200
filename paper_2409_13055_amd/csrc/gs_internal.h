// Internal definitions shared by the HIP kernels and the C-ABI entry points
// of libgs (gfx950).  Not part of the public interface (include/gs.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "gs.h"

namespace gs {

constexpr int kWave = 64;

// Binning windows: kWinSide x kWinSide tiles of one view, one wavefront lane
// per tile.
constexpr int kWinSide = 8;
constexpr int kWinShift = 3;

// Per-view geometry needed by the binning and raster kernels.
struct ViewGeom {
  int32_t W, H, TX, TY;
  int32_t tile_off, pix_off;
  int32_t WX, WY;    // binning windows per row / column
  int32_t win_off;   // global index of the view's first window
};
struct ViewTable {
  int32_t n_views;
  int32_t total_tiles;
  int32_t total_pixels;
  int32_t tile;
  int32_t total_windows;
  ViewGeom v[GS_MAX_VIEWS];
};

// Camera data needed by the projection kernels (plus derived constants).
struct CamF {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float centre[3];  // -R^T t
  float limx, limy; // frustum guard on x/z and y/z
  int32_t W, H;
};
struct CamTable {
  CamF c[GS_MAX_VIEWS];
};

// Status plumbing.
void set_error(const std::string& msg);
gs_status fail(gs_status s, const std::string& msg);
gs_status check_launch(const char* what);

gs_status validate_cams(const gs_camera* cams, int32_t n_views);
gs_status validate_opts(const gs_options* o);
gs_status validate_params(const gs_params* p);
ViewTable make_view_table(const gs_camera* cams, int32_t n_views, int32_t tile);
CamTable make_cam_table(const gs_camera* cams, int32_t n_views, const gs_options* o);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Round up to a multiple of 256 bytes (workspace sub-buffer alignment).
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Projected record field offsets (see gs_projected).
enum RecField { kMx = 0, kMy, kCa, kCb, kCc, kOp, kR, kG, kB, kDepth, kExtents, kFlags };

// Record word kExtents: the tile rect half-extents rx | ry << 16 (each at most
// kMaxExtent), 0 for a culled pair.
constexpr int kMaxExtent = 32767;
__host__ __device__ inline int ext_x(int packed) { return packed & 0xffff; }
__host__ __device__ inline int ext_y(int packed) { return packed >> 16; }

// Adam (the default 3DGS optimiser, Sec. IV-A).  1 - beta is formed in
// double on the host (forming it from the FP32 beta would be off by up to
// 1.3e-5 relative for beta = 0.999).  Shared by the standalone step and the
// projection backward fused with it, so both update a parameter bit for bit
// identically.
struct AdamCoef {
  double b1d, b2d;
  float b1, b2, omb1, omb2, eps;
};
__device__ __forceinline__ void adam_update(float& p, float g, float& m, float& v, const AdamCoef& c,
                                            float step_size, float inv_sqrt_bc2) {
  // every operation rounded on its own: where a multiply-add would be fused must not depend on
  // the kernel the update is inlined into
#pragma clang fp contract(off)
  m = c.b1 * m + c.omb1 * g;
  v = c.b2 * v + c.omb2 * g * g;
  p -= step_size * m / (sqrtf(v) * inv_sqrt_bc2 + c.eps);
}
// 1 / (1 - b1^t) and 1 / sqrt(1 - b2^t) for step t = step + 1, in double.
__device__ inline void adam_bias_factors(const AdamCoef& c, int32_t step, float& k1, float& k2) {
  const double st = (double)step + 1.0;
  k1 = (float)(1.0 / (1.0 - pow(c.b1d, st)));
  k2 = (float)(1.0 / sqrt(1.0 - pow(c.b2d, st)));
}
AdamCoef make_adam_coef(double beta1, double beta2, double eps);
gs_status validate_adam_hyper(double beta1, double beta2, double eps, const int32_t* d_step);
void launch_step_increment(int32_t* d_step, hipStream_t st);

// Which view owns global tile `gt` (views are few; linear scan).
__device__ inline int view_of_tile(const ViewTable& vt, int gt) {
  int v = 0;
#pragma unroll 1
  for (int u = 1; u < vt.n_views; ++u)
    if (vt.v[u].tile_off <= gt) v = u;
  return v;
}

// Tile rectangle of a splat with half-extents (rx, ry): [x0,x1) x [y0,y1),
// FP32 arithmetic in exactly this order (the bounds must agree bit for bit
// wherever they are computed).  It covers every pixel within extent - 1 of
// the mean.  The tile size B is 8, 16 or 32: 1/B is exact, so multiplying by
// it rounds exactly as the correctly rounded division by B does.
__device__ inline void tile_rect(float mx, float my, int rx, int ry, int B, int TX, int TY, int& x0, int& y0, int& x1,
                                 int& y1) {
  const float ex = (float)rx, ey = (float)ry, ib = ldexpf(1.0f, -__builtin_ctz((unsigned)B)), fb1 = (float)(B - 1);
  const float ax0 = floorf(__fmul_rn(__fsub_rn(mx, ex), ib));
  const float ax1 = floorf(__fmul_rn(__fadd_rn(__fadd_rn(mx, ex), fb1), ib));
  const float ay0 = floorf(__fmul_rn(__fsub_rn(my, ey), ib));
  const float ay1 = floorf(__fmul_rn(__fadd_rn(__fadd_rn(my, ey), fb1), ib));
  x0 = (int)fminf(fmaxf(ax0, 0.0f), (float)TX);
  x1 = (int)fminf(fmaxf(ax1, 0.0f), (float)TX);
  y0 = (int)fminf(fmaxf(ay0, 0.0f), (float)TY);
  y1 = (int)fminf(fmaxf(ay1, 0.0f), (float)TY);
}

}  // namespace gs
