// The photometric loss of eq. (2) with its SSIM term, and its gradient with
// respect to the rendered images.
//
// Reading of eq. (2) (printed garbled): per view, (1 - lambda) L1 +
// lambda (1 - SSIM), summed over views; SSIM as in the 3DGS loss: per channel,
// an 11 x 11 Gaussian window (sigma 1.5, normalised), zero-padded same-size
// filtering, C1 = 0.01^2, C2 = 0.03^2, the SSIM map averaged over the view's
// pixels and channels.
//
// With mu_x, mu_y, E[x^2], E[y^2], E[xy] the window sums around a pixel, the
// SSIM map is S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)
// (s_xx + s_yy + C2)).  Its gradient goes through the window sums: with
// A = dS/dmu_x, B = dS/dE[x^2], C = dS/dE[xy] per pixel, d mean(S) / dx =
// (W*A + 2 x W*B + y W*C) / n, W* the same zero-padded window (it is symmetric,
// so it is its own adjoint).  Two stencil kernels do that: the forward blurs
// the five maps of a tile (rows then columns, through LDS) and writes A, B, C;
// the backward blurs A, B, C and writes dL/dimage.  Both are bound by memory
// traffic and LDS, not by arithmetic.
#include <cmath>
#include <string>

#include "gs_internal.h"

namespace gs {

constexpr int kSsimTaps = 11, kSsimR = kSsimTaps / 2;
constexpr int kLossTH = 16, kLossTW = 64;  // output tile of a block (rows x columns)
constexpr int kLossThreads = 256;
constexpr int kLossInH = kLossTH + 2 * kSsimR, kLossInW = kLossTW + 2 * kSsimR;
constexpr int kLossPerThread = kLossTH * kLossTW / kLossThreads;  // output pixels per thread
static_assert(kLossPerThread * kLossThreads == kLossTH * kLossTW && kLossThreads % kLossTW == 0, "tile");

struct LossViews {
  int n_views, total_tiles;
  int W[GS_MAX_VIEWS], H[GS_MAX_VIEWS], TX[GS_MAX_VIEWS];
  long long pix_off[GS_MAX_VIEWS];
  int tile_off[GS_MAX_VIEWS + 1];
};

struct SsimConsts {
  float g[kSsimTaps];  // the 1D window (the 2D window is its outer product)
  float c1, c2, lam;
};

static LossViews make_loss_views(const gs_camera* cams, int32_t n_views) {
  LossViews lv{};
  lv.n_views = n_views;
  long long pix = 0;
  int tiles = 0;
  for (int v = 0; v < n_views; ++v) {
    lv.W[v] = cams[v].width;
    lv.H[v] = cams[v].height;
    lv.TX[v] = (cams[v].width + kLossTW - 1) / kLossTW;
    lv.pix_off[v] = pix;
    lv.tile_off[v] = tiles;
    tiles += lv.TX[v] * ((cams[v].height + kLossTH - 1) / kLossTH);
    pix += (long long)cams[v].width * cams[v].height;
  }
  lv.tile_off[n_views] = tiles;
  lv.total_tiles = tiles;
  return lv;
}

static SsimConsts make_ssim_consts(float lam) {
  SsimConsts k{};
  double g[kSsimTaps], sum = 0.0;
  for (int t = 0; t < kSsimTaps; ++t) {
    const double d = t - kSsimR;
    g[t] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[t];
  }
  for (int t = 0; t < kSsimTaps; ++t) k.g[t] = (float)(g[t] / sum);
  k.c1 = 0.01f * 0.01f;
  k.c2 = 0.03f * 0.03f;
  k.lam = lam;
  return k;
}

// The block's view and the tile's top-left pixel in it.
struct LossTile {
  int v, x0, y0, W, H;
  long long pix;  // pixel offset of the view
};
__device__ inline LossTile loss_tile(const LossViews& lv, int b) {
  int v = 0;
#pragma unroll 1
  for (int u = 1; u < lv.n_views; ++u)
    if (lv.tile_off[u] <= b) v = u;
  const int lt = b - lv.tile_off[v];
  LossTile t;
  t.v = v;
  t.W = lv.W[v];
  t.H = lv.H[v];
  t.x0 = (lt % lv.TX[v]) * kLossTW;
  t.y0 = (lt / lv.TX[v]) * kLossTH;
  t.pix = lv.pix_off[v];
  return t;
}

// The tile's input rectangle (with the halo, zero outside the image) of NMAP channel planes, read
// into registers (every load issued before any is used: the next channel's planes are in flight
// while the current one is filtered) and then stored to LDS.
constexpr int kHaloPerThread = (kLossInH * kLossInW + kLossThreads - 1) / kLossThreads;
template <int NMAP>
struct Halo {
  float v[NMAP][kHaloPerThread];
  __device__ inline void fetch(const float* const (&planes)[NMAP], const LossTile& t) {
    int at[kHaloPerThread];
#pragma unroll
    for (int k = 0; k < kHaloPerThread; ++k) {
      const int i = threadIdx.x + k * kLossThreads;
      const int r = i / kLossInW, c = i % kLossInW;
      const int y = t.y0 + r - kSsimR, x = t.x0 + c - kSsimR;
      const bool in = i < kLossInH * kLossInW && y >= 0 && y < t.H && x >= 0 && x < t.W;
      at[k] = in ? y * t.W + x : -1;
    }
#pragma unroll
    for (int m = 0; m < NMAP; ++m)
#pragma unroll
      for (int k = 0; k < kHaloPerThread; ++k) v[m][k] = at[k] >= 0 ? planes[m][at[k]] : 0.0f;
  }
  __device__ inline void put(float (*const (&dst)[NMAP])[kLossInW]) const {
#pragma unroll
    for (int k = 0; k < kHaloPerThread; ++k) {
      const int i = threadIdx.x + k * kLossThreads;
      if (i < kLossInH * kLossInW) {
        const int r = i / kLossInW, c = i % kLossInW;
#pragma unroll
        for (int m = 0; m < NMAP; ++m) dst[m][r][c] = v[m][k];
      }
    }
  }
};

__device__ inline size_t plane_of(const LossTile& t, int ch) {
  return (size_t)(3 * t.pix) + (size_t)ch * t.W * t.H;
}

__device__ inline float block_sum(float x, float* s_w) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  float t = 0.0f;
#pragma unroll
  for (int k = 0; k < kLossThreads / 64; ++k) t += s_w[k];
  __syncthreads();
  return t;
}

// Filtering through LDS: a thread takes two adjacent columns of a row in the row pass (its 12 inputs
// read once, as 8-byte pairs) and four consecutive rows of a column in the column pass (its 14
// inputs read once), instead of one LDS read per tap.
constexpr int kColPairs = kLossTW / 2;
constexpr int kRowRun = kLossPerThread;  // consecutive output rows per thread
static_assert(kLossTH == kRowRun * (kLossThreads / kLossTW), "column-pass rows");

__device__ inline void read_run12(const float* row, int c, float (&v)[kSsimTaps + 1]) {
#pragma unroll
  for (int m = 0; m < (kSsimTaps + 1) / 2; ++m) {
    const float2 p = *reinterpret_cast<const float2*>(row + c + 2 * m);
    v[2 * m] = p.x;
    v[2 * m + 1] = p.y;
  }
}

// Window sum down column `col` at output rows r0 .. r0 + kRowRun - 1 of one row-summed map.
__device__ inline void column_run(const float (*h)[kLossTW], int r0, int col, const SsimConsts& k,
                                  float (&out)[kRowRun]) {
  float v[kRowRun + kSsimTaps - 1];
#pragma unroll
  for (int q = 0; q < kRowRun + kSsimTaps - 1; ++q) v[q] = h[r0 + q][col];
#pragma unroll
  for (int p = 0; p < kRowRun; ++p) {
    float a = 0.0f;
#pragma unroll
    for (int q = 0; q < kSsimTaps; ++q) a = fmaf(k.g[q], v[p + q], a);
    out[p] = a;
  }
}

// Forward: per tile and channel, the five window sums, the SSIM map and its partials A, B, C
// (written for the backward), and the tile's sums of S and |x - y| (in a fixed order).
__global__ __launch_bounds__(kLossThreads) void k_ssim_fwd(LossViews lv, SsimConsts k,
                                                           const float* __restrict__ img,
                                                           const float* __restrict__ tgt,
                                                           float* __restrict__ ma, float* __restrict__ mb,
                                                           float* __restrict__ mc, float2* __restrict__ tile_part) {
  __shared__ __align__(16) float s_x[kLossInH][kLossInW];
  __shared__ __align__(16) float s_y[kLossInH][kLossInW];
  __shared__ __align__(16) float s_h[5][kLossInH][kLossTW];  // row sums of x, y, x^2, y^2, xy
  __shared__ float s_w[kLossThreads / 64];
  const LossTile t = loss_tile(lv, blockIdx.x);
  const int col = threadIdx.x % kLossTW, row0 = (threadIdx.x / kLossTW) * kRowRun;
  const bool want_grad = ma != nullptr;
  float ssum = 0.0f, l1sum = 0.0f;
  float (*const dst[2])[kLossInW] = {s_x, s_y};
  Halo<2> halo;
  {
    const float* const src[2] = {img + plane_of(t, 0), tgt + plane_of(t, 0)};
    halo.fetch(src, t);
  }
  for (int ch = 0; ch < 3; ++ch) {
    const size_t plane = plane_of(t, ch);
    halo.put(dst);
    __syncthreads();
    if (ch + 1 < 3) {
      const float* const src[2] = {img + plane_of(t, ch + 1), tgt + plane_of(t, ch + 1)};
      halo.fetch(src, t);
    }
    for (int i = threadIdx.x; i < kLossInH * kColPairs; i += kLossThreads) {
      const int r = i / kColPairs, c = 2 * (i % kColPairs);
      float xv[kSsimTaps + 1], yv[kSsimTaps + 1];
      read_run12(s_x[r], c, xv);
      read_run12(s_y[r], c, yv);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, a4 = 0.0f;
#pragma unroll
        for (int q = 0; q < kSsimTaps; ++q) {
          const float x = xv[u + q], y = yv[u + q], w = k.g[q], wx = w * x;
          a0 = fmaf(w, x, a0);
          a1 = fmaf(w, y, a1);
          a2 = fmaf(wx, x, a2);
          a3 = fmaf(w * y, y, a3);
          a4 = fmaf(wx, y, a4);
        }
        s_h[0][r][c + u] = a0;
        s_h[1][r][c + u] = a1;
        s_h[2][r][c + u] = a2;
        s_h[3][r][c + u] = a3;
        s_h[4][r][c + u] = a4;
      }
    }
    __syncthreads();
    float smx[kRowRun], smy[kRowRun], sexx[kRowRun], seyy[kRowRun], sexy[kRowRun];
    column_run(s_h[0], row0, col, k, smx);
    column_run(s_h[1], row0, col, k, smy);
    column_run(s_h[2], row0, col, k, sexx);
    column_run(s_h[3], row0, col, k, seyy);
    column_run(s_h[4], row0, col, k, sexy);
#pragma unroll
    for (int p = 0; p < kRowRun; ++p) {
      const int r = row0 + p;
      const float mx = smx[p], my = smy[p], exx = sexx[p], eyy = seyy[p], exy = sexy[p];
      const int y = t.y0 + r, x = t.x0 + col;
      if (y >= t.H || x >= t.W) continue;
      const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
      const float n1 = 2.0f * mx * my + k.c1, n2 = 2.0f * sxy + k.c2;
      const float d1 = mx * mx + my * my + k.c1, d2 = sxx + syy + k.c2;
      const float inv = 1.0f / (d1 * d2);
      const float s = n1 * n2 * inv;
      ssum += s;
      l1sum += fabsf(s_x[r + kSsimR][col + kSsimR] - s_y[r + kSsimR][col + kSsimR]);
      if (want_grad) {
        const size_t o = plane + (size_t)y * t.W + x;
        ma[o] = 2.0f * (my * (n2 - n1) - s * mx * (d2 - d1)) * inv;
        mb[o] = -s / d2;
        mc[o] = 2.0f * n1 * inv;
      }
    }
    __syncthreads();  // the next channel overwrites the LDS planes
  }
  ssum = block_sum(ssum, s_w);
  l1sum = block_sum(l1sum, s_w);
  if (threadIdx.x == 0) tile_part[blockIdx.x] = make_float2(ssum, l1sum);
}

// Backward: dL/dx = (1 - lambda) sign(x - y) / n - lambda (W*A + 2 x W*B + y W*C) / n per pixel,
// n = 3 H W of its view.
__global__ __launch_bounds__(kLossThreads) void k_ssim_bwd(LossViews lv, SsimConsts k,
                                                           const float* __restrict__ img,
                                                           const float* __restrict__ tgt,
                                                           const float* __restrict__ ma,
                                                           const float* __restrict__ mb,
                                                           const float* __restrict__ mc,
                                                           float* __restrict__ dl) {
  __shared__ __align__(16) float s_m[3][kLossInH][kLossInW];
  __shared__ __align__(16) float s_h[3][kLossInH][kLossTW];
  const LossTile t = loss_tile(lv, blockIdx.x);
  const int col = threadIdx.x % kLossTW, row0 = (threadIdx.x / kLossTW) * kRowRun;
  const float inv_n = 1.0f / (3.0f * (float)t.W * (float)t.H);
  const float w_l1 = (1.0f - k.lam) * inv_n, w_s = k.lam * inv_n;
  float (*const dst[3])[kLossInW] = {s_m[0], s_m[1], s_m[2]};
  Halo<3> halo;
  {
    const size_t p0 = plane_of(t, 0);
    const float* const src[3] = {ma + p0, mb + p0, mc + p0};
    halo.fetch(src, t);
  }
  for (int ch = 0; ch < 3; ++ch) {
    const size_t plane = plane_of(t, ch);
    halo.put(dst);
    __syncthreads();
    if (ch + 1 < 3) {
      const size_t pn = plane_of(t, ch + 1);
      const float* const src[3] = {ma + pn, mb + pn, mc + pn};
      halo.fetch(src, t);
    }
    for (int i = threadIdx.x; i < kLossInH * kColPairs; i += kLossThreads) {
      const int r = i / kColPairs, c = 2 * (i % kColPairs);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        float v[kSsimTaps + 1];
        read_run12(s_m[m][r], c, v);
        float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
        for (int q = 0; q < kSsimTaps; ++q) {
          a0 = fmaf(k.g[q], v[q], a0);
          a1 = fmaf(k.g[q], v[q + 1], a1);
        }
        s_h[m][r][c] = a0;
        s_h[m][r][c + 1] = a1;
      }
    }
    __syncthreads();
    float sga[kRowRun], sgb[kRowRun], sgc[kRowRun];
    column_run(s_h[0], row0, col, k, sga);
    column_run(s_h[1], row0, col, k, sgb);
    column_run(s_h[2], row0, col, k, sgc);
#pragma unroll
    for (int p = 0; p < kRowRun; ++p) {
      const int r = row0 + p;
      const float ga = sga[p], gb = sgb[p], gc = sgc[p];
      const int y = t.y0 + r, x = t.x0 + col;
      if (y >= t.H || x >= t.W) continue;
      const size_t o = plane + (size_t)y * t.W + x;
      const float xv = img[o], yv = tgt[o], d = xv - yv;
      const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
      dl[o] = w_l1 * sgn - w_s * fmaf(yv, gc, fmaf(2.0f * xv, gb, ga));
    }
    __syncthreads();
  }
}

// Per view, in a fixed order: loss = (1 - lambda) L1 + lambda (1 - SSIM).
__global__ __launch_bounds__(kLossThreads) void k_photometric_reduce(LossViews lv, SsimConsts k,
                                                                    const float2* __restrict__ tile_part,
                                                                    float* __restrict__ loss_out) {
  __shared__ float s_w[kLossThreads / 64];
  const int v = blockIdx.x;
  float ss = 0.0f, l1 = 0.0f;
  for (int b = lv.tile_off[v] + (int)threadIdx.x; b < lv.tile_off[v + 1]; b += kLossThreads) {
    const float2 p = tile_part[b];
    ss += p.x;
    l1 += p.y;
  }
  ss = block_sum(ss, s_w);
  l1 = block_sum(l1, s_w);
  if (threadIdx.x == 0) {
    const float n = 3.0f * (float)lv.W[v] * (float)lv.H[v];
    loss_out[v] = (1.0f - k.lam) * (l1 / n) + k.lam * (1.0f - ss / n);
  }
}

struct LossWorkspace {
  size_t off_a, off_b, off_c, off_part, bytes;
};
static LossWorkspace loss_workspace(const LossViews& lv, long long total_pixels, bool grad) {
  LossWorkspace w{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += (b + 255) / 256 * 256;
    return at;
  };
  const size_t maps = grad ? sizeof(float) * 3 * (size_t)total_pixels : 0;
  w.off_a = take(maps);
  w.off_b = take(maps);
  w.off_c = take(maps);
  w.off_part = take(sizeof(float2) * (size_t)lv.total_tiles);
  w.bytes = o;
  return w;
}

}  // namespace gs

extern "C" gs_status gs_photometric_loss_workspace_size(const gs_camera* cams, int32_t n_views, size_t* bytes) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if (!bytes) return fail(GS_ERR_INVALID_VALUE, "bytes is NULL");
  long long px = 0;
  for (int v = 0; v < n_views; ++v) px += (long long)cams[v].width * cams[v].height;
  *bytes = loss_workspace(make_loss_views(cams, n_views), px, true).bytes;
  return GS_OK;
}

extern "C" gs_status gs_photometric_loss(const gs_camera* cams, int32_t n_views, const float* image,
                                         const float* target, float lambda, float* loss_out, float* dl_dimage,
                                         void* workspace, size_t workspace_bytes, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if (!image || !target) return fail(GS_ERR_INVALID_VALUE, "image and target are required");
  if (!loss_out && !dl_dimage) return fail(GS_ERR_INVALID_VALUE, "nothing to compute: loss_out and dl_dimage are NULL");
  if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(GS_ERR_INVALID_VALUE, "lambda must be in [0, 1]");
  const LossViews lv = make_loss_views(cams, n_views);
  long long px = 0;
  for (int v = 0; v < n_views; ++v) px += (long long)cams[v].width * cams[v].height;
  const bool grad = dl_dimage != nullptr;
  const LossWorkspace w = loss_workspace(lv, px, grad);
  if (!workspace || workspace_bytes < w.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(w.bytes) + " bytes");
  char* ws = static_cast<char*>(workspace);
  float* ma = grad ? reinterpret_cast<float*>(ws + w.off_a) : nullptr;
  float* mb = grad ? reinterpret_cast<float*>(ws + w.off_b) : nullptr;
  float* mc = grad ? reinterpret_cast<float*>(ws + w.off_c) : nullptr;
  float2* part = reinterpret_cast<float2*>(ws + w.off_part);
  const SsimConsts k = make_ssim_consts(lambda);
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_ssim_fwd, dim3((unsigned)lv.total_tiles), dim3(kLossThreads), 0, st, lv, k, image, target, ma,
                     mb, mc, part);
  if (loss_out)
    hipLaunchKernelGGL(k_photometric_reduce, dim3((unsigned)n_views), dim3(kLossThreads), 0, st, lv, k, part,
                       loss_out);
  if (grad)
    hipLaunchKernelGGL(k_ssim_bwd, dim3((unsigned)lv.total_tiles), dim3(kLossThreads), 0, st, lv, k, image, target, ma,
                       mb, mc, dl_dimage);
  return check_launch("photometric loss");
}
