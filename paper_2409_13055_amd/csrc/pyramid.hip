// Gaussian pyramid of the ground-truth images for coarse-to-fine training
// (Sec. III-B, after Photo-SLAM): each level smooths and halves the one
// below it.
//
// Reading (the paper names the technique but not its filter): one level is
// Burt and Adelson's REDUCE step, the separable binomial window
// (1, 4, 6, 4, 1) / 16 centred on every second pixel, output size
// ceil(W/2) x ceil(H/2), borders reflected without repeating the edge pixel.
// Output pixel x' samples input index 2 x', so a level's camera has
// fx' = fx / 2, cx' = cx / 2 + 1/4 (index coordinates put a camera-frame
// point at fx x/z + cx - 1/2), likewise in y.
//
// The kernel is bound by HBM traffic (one read of the input, a quarter of it
// written): a block stages the reflected input rectangle of a 16 x 64 output
// tile in LDS with coalesced loads, filters its rows at the even columns
// (8-byte LDS reads, conflict-free), then its columns at the even rows, for
// the three channels in turn with the next channel's loads in flight.
#include <string>

#include "gs_internal.h"

namespace gs {

constexpr int kPyrTH = 16, kPyrTW = 64;  // output tile of a block (rows x columns)
constexpr int kPyrThreads = 256;
constexpr int kPyrInH = 2 * kPyrTH + 3, kPyrInW = 2 * kPyrTW + 3;  // input rectangle, 2-pixel halo
constexpr int kPyrLd = kPyrInW + 1;  // even LDS row stride: the row pass reads 8-byte pairs
constexpr int kPyrLoads = (kPyrInH * kPyrInW + kPyrThreads - 1) / kPyrThreads;
constexpr int kPyrGroups = kPyrThreads / kPyrTW;  // lanes per output column: row groups of a block
static_assert(kPyrThreads % kPyrTW == 0 && kPyrTH % kPyrGroups == 0, "tile");

struct PyrViews {
  int n_views;
  int W[GS_MAX_VIEWS], H[GS_MAX_VIEWS], W2[GS_MAX_VIEWS], H2[GS_MAX_VIEWS], TX[GS_MAX_VIEWS];
  long long src_off[GS_MAX_VIEWS], dst_off[GS_MAX_VIEWS];  // first float of the view
  int tile_off[GS_MAX_VIEWS + 1];
};

static PyrViews make_pyr_views(const gs_camera* cams, int32_t n_views, long long* src_floats, long long* dst_floats) {
  PyrViews pv{};
  pv.n_views = n_views;
  long long s = 0, d = 0;
  int tiles = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = cams[v].width, H = cams[v].height, W2 = (W + 1) / 2, H2 = (H + 1) / 2;
    pv.W[v] = W;
    pv.H[v] = H;
    pv.W2[v] = W2;
    pv.H2[v] = H2;
    pv.TX[v] = (W2 + kPyrTW - 1) / kPyrTW;
    pv.src_off[v] = s;
    pv.dst_off[v] = d;
    pv.tile_off[v] = tiles;
    tiles += pv.TX[v] * ((H2 + kPyrTH - 1) / kPyrTH);
    s += 3LL * W * H;
    d += 3LL * W2 * H2;
  }
  pv.tile_off[n_views] = tiles;
  *src_floats = s;
  *dst_floats = d;
  return pv;
}

// Index i of an axis of n samples reflected about the end samples (not repeated).  The rows and
// columns that valid outputs read lie in [-2, n + 1]; indices past n + 1 (the unused part of a
// ragged tile) are first clamped to n + 1, so every returned index is in [0, n).
__device__ inline int reflect101(int i, int n) {
  if (n == 1) return 0;
  i = min(i, n + 1);
  i = i < 0 ? -i : i;
  i = i >= n ? 2 * n - 2 - i : i;
  return i < 0 ? -i : i;
}

__device__ inline float taps5(float a, float b, float c, float d, float e) {
  return fmaf(0.0625f, a + e, fmaf(0.25f, b + d, 0.375f * c));
}

__global__ __launch_bounds__(kPyrThreads) void k_pyramid_reduce(PyrViews pv, const float* __restrict__ src,
                                                                  float* __restrict__ dst) {
  __shared__ __align__(16) float s_in[kPyrInH][kPyrLd];
  __shared__ float s_row[kPyrInH][kPyrTW];
  const int b = blockIdx.x, tid = threadIdx.x;
  int v = 0;
#pragma unroll 1
  for (int u = 1; u < pv.n_views; ++u)
    if (pv.tile_off[u] <= b) v = u;
  const int W = pv.W[v], H = pv.H[v], W2 = pv.W2[v], H2 = pv.H2[v];
  const int lt = b - pv.tile_off[v];
  const int ox0 = (lt % pv.TX[v]) * kPyrTW, oy0 = (lt / pv.TX[v]) * kPyrTH;
  const size_t plane = (size_t)W * H, plane2 = (size_t)W2 * H2;
  const float* in = src + pv.src_off[v];
  float* out = dst + pv.dst_off[v];

  // offsets in a channel plane of the input rectangle, rows 2 oy0 - 2 .. 2 oy0 + 2 TH and columns
  // 2 ox0 - 2 .. 2 ox0 + 2 TW (reflected); -1 past the rectangle
  int at[kPyrLoads];
#pragma unroll
  for (int k = 0; k < kPyrLoads; ++k) {
    const int i = tid + k * kPyrThreads;
    const int r = i / kPyrInW, c = i % kPyrInW;
    at[k] = i < kPyrInH * kPyrInW ? reflect101(2 * oy0 - 2 + r, H) * W + reflect101(2 * ox0 - 2 + c, W) : -1;
  }
  // the three channels in turn; the next channel's loads are issued before the current one is filtered
  float val[kPyrLoads];
#pragma unroll
  for (int k = 0; k < kPyrLoads; ++k) val[k] = at[k] >= 0 ? in[at[k]] : 0.0f;
  const int lx = tid % kPyrTW, g = tid / kPyrTW, ox = ox0 + lx;
#pragma unroll 1
  for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
    for (int k = 0; k < kPyrLoads; ++k) {
      const int i = tid + k * kPyrThreads;
      if (i < kPyrInH * kPyrInW) s_in[i / kPyrInW][i % kPyrInW] = val[k];
    }
    __syncthreads();
    if (ch < 2) {
      const float* next = in + (ch + 1) * plane;
#pragma unroll
      for (int k = 0; k < kPyrLoads; ++k) val[k] = at[k] >= 0 ? next[at[k]] : 0.0f;
    }
    // rows: the window at input column 2 x (staged column 2 x + 2) for every staged row
#pragma unroll
    for (int j = 0; j < (kPyrInH + kPyrGroups - 1) / kPyrGroups; ++j) {
      const int r = g + j * kPyrGroups;
      if (r >= kPyrInH) break;
      const float2 p0 = *reinterpret_cast<const float2*>(&s_in[r][2 * lx]);
      const float2 p1 = *reinterpret_cast<const float2*>(&s_in[r][2 * lx + 2]);
      const float p2 = s_in[r][2 * lx + 4];
      s_row[r][lx] = taps5(p0.x, p0.y, p1.x, p1.y, p2);
    }
    __syncthreads();
    // columns: the window at input row 2 y (staged row 2 y + 2); the next channel's stores to
    // s_in are ordered after these reads' row pass by the barrier above, and the next row pass
    // after them by the barrier that follows those stores
#pragma unroll
    for (int j = 0; j < kPyrTH / kPyrGroups; ++j) {
      const int y = g + j * kPyrGroups, oy = oy0 + y;
      const float o = taps5(s_row[2 * y][lx], s_row[2 * y + 1][lx], s_row[2 * y + 2][lx], s_row[2 * y + 3][lx],
                            s_row[2 * y + 4][lx]);
      if (ox < W2 && oy < H2) out[ch * plane2 + (size_t)oy * W2 + ox] = o;
    }
  }
}

}  // namespace gs

extern "C" gs_status gs_pyramid_camera(const gs_camera* cam, int32_t levels, gs_camera* out) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cam, 1)) != GS_OK) return s;
  if (!out) return fail(GS_ERR_INVALID_VALUE, "out is NULL");
  if (levels < 0 || levels > 15) return fail(GS_ERR_INVALID_VALUE, "levels must be in [0, 15]");
  gs_camera c = *cam;
  for (int l = 0; l < levels; ++l) {
    c.fx *= 0.5f;
    c.fy *= 0.5f;
    c.cx = c.cx * 0.5f + 0.25f;
    c.cy = c.cy * 0.5f + 0.25f;
    c.width = (c.width + 1) / 2;
    c.height = (c.height + 1) / 2;
  }
  *out = c;
  return GS_OK;
}

extern "C" gs_status gs_pyramid_reduce(const gs_camera* cams, int32_t n_views, const float* src, float* dst,
                                       void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if (!src || !dst) return fail(GS_ERR_INVALID_VALUE, "src and dst are required");
  long long ns = 0, nd = 0;
  const PyrViews pv = make_pyr_views(cams, n_views, &ns, &nd);
  const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), s1 = s0 + (uintptr_t)ns * sizeof(float);
  const uintptr_t d0 = reinterpret_cast<uintptr_t>(dst), d1 = d0 + (uintptr_t)nd * sizeof(float);
  if (s0 < d1 && d0 < s1) return fail(GS_ERR_INVALID_VALUE, "src and dst overlap");
  hipLaunchKernelGGL(k_pyramid_reduce, dim3((unsigned)pv.tile_off[n_views]), dim3(kPyrThreads), 0,
                     as_stream(stream), pv, src, dst);
  return check_launch("pyramid reduce");
}
