// Point-cloud densification of a keyframe (Sec. III-A) and the
// initialisation of new Gaussians from it (Sec. III-B).
//
// The paper triangulates the image with the tracked pixels as vertices
// (Delaunay), gives the pixels of low-gradient regions the mean depth of their
// triangle's vertices, and starts new Gaussians at the points with their
// colour.  The triangulation is host code (delaunay.cpp).  Readings:
//  - a pixel belongs to the triangle whose closed interior holds it, an edge
//    shared by two triangles going to one of them: edge a -> b of a triangle
//    of positive orientation is its own when b.y > a.y, or b.y == a.y and
//    b.x < a.x (exact integer tests); a tracked pixel keeps its own depth;
//  - low gradient: grey = (r + g + b) / 3, central differences (one-sided at
//    the border), gx^2 + gy^2 < tau^2, every step an FP32 operation without
//    contraction, so the decision is the reference's bit for bit;
//  - one new Gaussian per pixel with a depth on the grid of stride `stride`
//    (tracked pixels always), in row-major pixel order: mean = the pixel's
//    index coordinate unprojected at its depth, sh_dc = (colour - 1/2) / SH_C0,
//    identity rotation, opacity 0.1 (the 3DGS initial opacity), isotropic
//    scale stride * depth / fx (the pixel footprint), higher bands 0.
// The per-pixel kernels are bound by HBM traffic; the triangle fill walks each
// triangle's bounding box with one block per triangle.
#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "gs_internal.h"

namespace gs {

// ---------------------------------------------------------------- kernels
constexpr int kPcThreads = 256;
constexpr int kPcScanThreads = 1024;

__global__ __launch_bounds__(kPcThreads) void k_pc_clear(int64_t n_px, float* __restrict__ depth,
                                                          uint8_t* __restrict__ tracked) {
  const int64_t i = (int64_t)blockIdx.x * kPcThreads + threadIdx.x;
  if (i < n_px) {
    depth[i] = 0.0f;
    tracked[i] = 0;
  }
}

__global__ __launch_bounds__(kPcThreads) void k_pc_tracked(int n, int W, int H, const int32_t* __restrict__ xy,
                                                            const float* __restrict__ d, float* __restrict__ depth,
                                                            uint8_t* __restrict__ tracked) {
  const int i = blockIdx.x * kPcThreads + threadIdx.x;
  if (i >= n) return;
  const int x = xy[2 * i], y = xy[2 * i + 1];
  if (x < 0 || y < 0 || x >= W || y >= H) return;  // outside the image: not a pixel of it
  const int64_t p = (int64_t)y * W + x;
  depth[p] = d[i];
  tracked[p] = 1;
}

// grey level of pixel (x, y): (r + g + b) / 3 in FP32, no contraction
__device__ inline float grey_at(const float* __restrict__ img, int64_t plane, int64_t p) {
  return __fdiv_rn(__fadd_rn(__fadd_rn(img[p], img[plane + p]), img[2 * plane + p]), 3.0f);
}

__device__ inline bool low_gradient(const float* __restrict__ img, int W, int H, int x, int y, float tau2) {
  const int64_t plane = (int64_t)W * H, row = (int64_t)y * W;
  float gx = 0.0f, gy = 0.0f;
  if (W > 1) {
    if (x == 0) gx = __fsub_rn(grey_at(img, plane, row + 1), grey_at(img, plane, row));
    else if (x == W - 1) gx = __fsub_rn(grey_at(img, plane, row + x), grey_at(img, plane, row + x - 1));
    else gx = __fmul_rn(__fsub_rn(grey_at(img, plane, row + x + 1), grey_at(img, plane, row + x - 1)), 0.5f);
  }
  if (H > 1) {
    if (y == 0) gy = __fsub_rn(grey_at(img, plane, W + x), grey_at(img, plane, x));
    else if (y == H - 1) gy = __fsub_rn(grey_at(img, plane, row + x), grey_at(img, plane, row - W + x));
    else gy = __fmul_rn(__fsub_rn(grey_at(img, plane, row + W + x), grey_at(img, plane, row - W + x)), 0.5f);
  }
  return __fadd_rn(__fmul_rn(gx, gx), __fmul_rn(gy, gy)) < tau2;
}

// One block per triangle: the pixels of its bounding box it owns, not tracked and of low gradient,
// get the mean depth of its vertices.  Every pixel has at most one owner, so the stores do not race.
__global__ __launch_bounds__(kPcThreads) void k_pc_fill(int n_tris, int n, int W, int H, const int32_t* __restrict__ xy,
                                                         const float* __restrict__ d, const int32_t* __restrict__ tris,
                                                         const float* __restrict__ img, float tau2,
                                                         float* __restrict__ depth,
                                                         const uint8_t* __restrict__ tracked) {
  const int t = blockIdx.x;
  if (t >= n_tris) return;
  int v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
  for (int k = 0; k < 3; ++k)
    if (v[k] < 0 || v[k] >= n) return;  // not a triangle of these points
  int64_t X[3], Y[3];
  for (int k = 0; k < 3; ++k) {
    X[k] = xy[2 * v[k]];
    Y[k] = xy[2 * v[k] + 1];
  }
  if ((X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]) < 0) {
    int64_t tx = X[1], ty = Y[1];
    X[1] = X[2];
    Y[1] = Y[2];
    X[2] = tx;
    Y[2] = ty;
  }
  bool own[3];
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3;
    own[k] = Y[k1] > Y[k] || (Y[k1] == Y[k] && X[k1] < X[k]);
  }
  const float mean = __fdiv_rn(__fadd_rn(__fadd_rn(d[v[0]], d[v[1]]), d[v[2]]), 3.0f);
  const int x0 = (int)max((int64_t)0, min(X[0], min(X[1], X[2])));
  const int x1 = (int)min((int64_t)W - 1, max(X[0], max(X[1], X[2])));
  const int y0 = (int)max((int64_t)0, min(Y[0], min(Y[1], Y[2])));
  const int y1 = (int)min((int64_t)H - 1, max(Y[0], max(Y[1], Y[2])));
  const int bw = x1 - x0 + 1;
  const int64_t cnt = (int64_t)bw * (y1 - y0 + 1);
  for (int64_t q = threadIdx.x; q < cnt; q += kPcThreads) {
    const int x = x0 + (int)(q % bw), y = y0 + (int)(q / bw);
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3;
      const int64_t e = (X[k1] - X[k]) * (y - Y[k]) - (Y[k1] - Y[k]) * (x - X[k]);
      inside = inside && (e > 0 || (e == 0 && own[k]));
    }
    if (!inside) continue;
    const int64_t p = (int64_t)y * W + x;
    if (tracked[p] || !low_gradient(img, W, H, x, y, tau2)) continue;
    depth[p] = mean;
  }
}

// Pixels that start a Gaussian: a depth, and on the stride grid or tracked.
__device__ inline bool pc_used(int64_t p, int64_t n_px, int W, int stride, const float* depth,
                               const uint8_t* tracked) {
  if (p >= n_px) return false;
  const int x = (int)(p % W), y = (int)(p / W);
  return depth[p] > 0.0f && ((x % stride == 0 && y % stride == 0) || tracked[p]);
}

__device__ inline int block_rank(bool f, int& total) {
  __shared__ int s_w[kPcThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const unsigned long long m = __ballot(f);
  if (lane == 0) s_w[w] = __popcll(m);
  __syncthreads();
  int before = 0;
  total = 0;
  for (int u = 0; u < kPcThreads / kWave; ++u) {
    before += u < w ? s_w[u] : 0;
    total += s_w[u];
  }
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  return before + __popcll(m & below);
}

__global__ __launch_bounds__(kPcThreads) void k_pc_count(int64_t n_px, int W, int stride,
                                                          const float* __restrict__ depth,
                                                          const uint8_t* __restrict__ tracked,
                                                          int32_t* __restrict__ block_counts) {
  const int64_t p = (int64_t)blockIdx.x * kPcThreads + threadIdx.x;
  int total;
  block_rank(pc_used(p, n_px, W, stride, depth, tracked), total);
  if (threadIdx.x == 0) block_counts[blockIdx.x] = total;
}

__global__ __launch_bounds__(kPcScanThreads) void k_pc_scan(int64_t nb, const int32_t* __restrict__ counts,
                                                             int32_t* __restrict__ offs, int32_t* __restrict__ total) {
  __shared__ int s[kPcScanThreads];
  const int t = threadIdx.x;
  const int64_t per = (nb + kPcScanThreads - 1) / kPcScanThreads;
  const int64_t b0 = (int64_t)t * per, b1 = b0 + per < nb ? b0 + per : nb;
  int local = 0;
  for (int64_t b = b0; b < b1; ++b) local += counts[b];
  s[t] = local;
  __syncthreads();
  for (int o = 1; o < kPcScanThreads; o <<= 1) {
    const int x = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  int run = s[t] - local;
  for (int64_t b = b0; b < b1; ++b) {
    offs[b] = run;
    run += counts[b];
  }
  if (t == kPcScanThreads - 1) *total = s[t];
}

struct PcInit {
  float R[9], t[3], fx, fy, cx, cy, logit0, inv_c0;
  int W, stride, rest;
};

__global__ __launch_bounds__(kPcThreads) void k_pc_write(int64_t n_px, PcInit c, const float* __restrict__ depth,
                                                          const uint8_t* __restrict__ tracked,
                                                          const float* __restrict__ img,
                                                          const int32_t* __restrict__ offs, int64_t n_out,
                                                          float* __restrict__ means, float* __restrict__ log_scales,
                                                          float* __restrict__ quats, float* __restrict__ logits,
                                                          float* __restrict__ sh_dc, float* __restrict__ sh_rest) {
  const int64_t p = (int64_t)blockIdx.x * kPcThreads + threadIdx.x;
  const bool used = pc_used(p, n_px, c.W, c.stride, depth, tracked);
  int total;
  const int r = block_rank(used, total);
  if (!used) return;
  const int64_t j = offs[blockIdx.x] + r;
  if (j >= n_out) return;
  const float z = depth[p];
  const float x = (float)(p % c.W), y = (float)(p / c.W);
  // camera frame: index coordinate u = fx X/Z + cx - 1/2
  const float pc[3] = {(x - c.cx + 0.5f) / c.fx * z, (y - c.cy + 0.5f) / c.fy * z, z};
  const float q[3] = {pc[0] - c.t[0], pc[1] - c.t[1], pc[2] - c.t[2]};
  for (int k = 0; k < 3; ++k)  // world = R^T (pc - t)
    means[3 * j + k] = fmaf(c.R[k], q[0], fmaf(c.R[3 + k], q[1], c.R[6 + k] * q[2]));
  const float ls = logf((float)c.stride * z / c.fx);
  for (int k = 0; k < 3; ++k) log_scales[3 * j + k] = ls;
  quats[4 * j] = 1.0f;
  quats[4 * j + 1] = quats[4 * j + 2] = quats[4 * j + 3] = 0.0f;
  logits[j] = c.logit0;
  const int64_t plane = n_px;
  for (int k = 0; k < 3; ++k) sh_dc[3 * j + k] = (img[k * plane + p] - 0.5f) * c.inv_c0;
  for (int k = 0; k < c.rest; ++k) sh_rest[j * c.rest + k] = 0.0f;
}

struct PcWs {
  int32_t* counts;
  int32_t* offs;
  size_t bytes;
};
static PcWs pc_ws(void* base, int64_t n_px) {
  const int64_t nb = (n_px + kPcThreads - 1) / kPcThreads;
  char* p = static_cast<char*>(base);
  PcWs w{};
  w.counts = reinterpret_cast<int32_t*>(p);
  w.offs = reinterpret_cast<int32_t*>(p + align256((size_t)nb * 4));
  w.bytes = 2 * align256((size_t)nb * 4);
  return w;
}

}  // namespace gs

extern "C" gs_status gs_densify_depth(const gs_camera* cam, const int32_t* xy, const float* depth, int32_t n,
                                      const int32_t* tris, int32_t n_tris, const float* image, float tau,
                                      float* depth_map, uint8_t* tracked, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cam, 1)) != GS_OK) return s;
  if (n < 0 || n_tris < 0) return fail(GS_ERR_INVALID_VALUE, "n and n_tris must be >= 0");
  if ((n > 0 && (!xy || !depth)) || (n_tris > 0 && !tris) || !image || !depth_map || !tracked)
    return fail(GS_ERR_INVALID_VALUE, "a required array is NULL");
  if (!(tau >= 0.0f) || !std::isfinite(tau)) return fail(GS_ERR_INVALID_VALUE, "tau must be finite and >= 0");
  const int W = cam->width, H = cam->height;
  const int64_t n_px = (int64_t)W * H;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_pc_clear, dim3((unsigned)((n_px + kPcThreads - 1) / kPcThreads)), dim3(kPcThreads), 0, st,
                     n_px, depth_map, tracked);
  if (n > 0)
    hipLaunchKernelGGL(k_pc_tracked, dim3((unsigned)((n + kPcThreads - 1) / kPcThreads)), dim3(kPcThreads), 0, st, n,
                       W, H, xy, depth, depth_map, tracked);
  if (n_tris > 0)
    hipLaunchKernelGGL(k_pc_fill, dim3((unsigned)n_tris), dim3(kPcThreads), 0, st, n_tris, n, W, H, xy, depth, tris,
                       image, tau * tau, depth_map, tracked);
  return check_launch("densify depth");
}

extern "C" gs_status gs_init_gaussians_workspace_size(const gs_camera* cam, size_t* bytes) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cam, 1)) != GS_OK) return s;
  if (!bytes) return fail(GS_ERR_INVALID_VALUE, "bytes is NULL");
  *bytes = pc_ws(nullptr, (int64_t)cam->width * cam->height).bytes;
  return GS_OK;
}

extern "C" gs_status gs_init_gaussians_count(const gs_camera* cam, const float* depth_map, const uint8_t* tracked,
                                             int32_t stride, int32_t* d_count, void* workspace,
                                             size_t workspace_bytes, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cam, 1)) != GS_OK) return s;
  if (!depth_map || !tracked || !d_count) return fail(GS_ERR_INVALID_VALUE, "a required array is NULL");
  if (stride < 1) return fail(GS_ERR_INVALID_VALUE, "stride must be >= 1");
  const int64_t n_px = (int64_t)cam->width * cam->height;
  const PcWs w = pc_ws(workspace, n_px);
  if (!workspace || workspace_bytes < w.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(w.bytes) + " bytes");
  const int64_t nb = (n_px + kPcThreads - 1) / kPcThreads;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_pc_count, dim3((unsigned)nb), dim3(kPcThreads), 0, st, n_px, cam->width, stride, depth_map,
                     tracked, w.counts);
  hipLaunchKernelGGL(k_pc_scan, dim3(1), dim3(kPcScanThreads), 0, st, nb, w.counts, w.offs, d_count);
  return check_launch("initialisation count");
}

extern "C" gs_status gs_init_gaussians(const gs_camera* cam, const float* depth_map, const uint8_t* tracked,
                                       const float* image, int32_t stride, int32_t sh_degree, int64_t n_out,
                                       const gs_grads* out, const void* workspace, size_t workspace_bytes,
                                       void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cam, 1)) != GS_OK) return s;
  if (!depth_map || !tracked || !image) return fail(GS_ERR_INVALID_VALUE, "a required array is NULL");
  if (stride < 1) return fail(GS_ERR_INVALID_VALUE, "stride must be >= 1");
  if (sh_degree < 0 || sh_degree > GS_MAX_SH_DEGREE) return fail(GS_ERR_INVALID_VALUE, "sh_degree must be in [0, 3]");
  const int64_t n_px = (int64_t)cam->width * cam->height;
  if (n_out < 0 || n_out > n_px) return fail(GS_ERR_INVALID_VALUE, "n_out must be in [0, W H]");
  const PcWs w = pc_ws(const_cast<void*>(workspace), n_px);
  if (!workspace || workspace_bytes < w.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(w.bytes) + " bytes");
  if (n_out == 0) return GS_OK;
  if (!out || !out->means || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh_dc ||
      (sh_degree > 0 && !out->sh_rest))
    return fail(GS_ERR_INVALID_VALUE, "an output array is NULL");
  PcInit c{};
  for (int k = 0; k < 9; ++k) c.R[k] = cam->R[k];
  for (int k = 0; k < 3; ++k) c.t[k] = cam->t[k];
  c.fx = cam->fx;
  c.fy = cam->fy;
  c.cx = cam->cx;
  c.cy = cam->cy;
  c.logit0 = (float)std::log(0.1 / 0.9);
  c.inv_c0 = (float)(2.0 * std::sqrt(M_PI));  // 1 / SH_C0, SH_C0 = 1 / (2 sqrt(pi))
  c.W = cam->width;
  c.stride = stride;
  c.rest = 3 * ((sh_degree + 1) * (sh_degree + 1) - 1);
  const int64_t nb = (n_px + kPcThreads - 1) / kPcThreads;
  hipLaunchKernelGGL(k_pc_write, dim3((unsigned)nb), dim3(kPcThreads), 0, as_stream(stream), n_px, c, depth_map,
                     tracked, image, w.offs, n_out, out->means, out->log_scales, out->quats, out->opacity_logits,
                     out->sh_dc, out->sh_rest);
  return check_launch("initialise Gaussians");
}
