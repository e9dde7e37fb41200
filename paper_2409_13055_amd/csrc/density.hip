// Adaptive density control of the Gaussian map (Sec. III-B): AbsGS
// densification (Gaussians whose homodirectional view-space position gradient
// is high are split when large and cloned when small, with the 3DGS split and
// clone parameters the paper keeps) and pruning of low-opacity Gaussians.
//
// Readings (the paper names the method, not its formulas):
//  - statistics as in 3DGS, one observation per (view, Gaussian) pair whose
//    Gaussian touches a tile of the view: the view-space gradient is the
//    mean's gradient in normalised device units, (W/2) dL/dmx and
//    (H/2) dL/dmy; the homodirectional gradient (AbsGS) takes the sums of the
//    per-pixel magnitudes instead (gs_raster_bwd_abs); the Euclidean norm of
//    each goes into an accumulator and the pair adds 1 to a count;
//  - selected: abs_accum >= tau * count (FP32 product), count > 0;
//  - selected and max log-scale > log(percent_dense * extent): split into two
//    children with means mu + R (s * eps) (eps standard normal, passed in) and
//    log-scales reduced by log(split_scale_div); selected otherwise: cloned;
//  - logit below logit(min_opacity): pruned, with no clone or split;
//  - new order: kept originals, clones, first children, second children, each
//    in the original order; Adam moments kept for originals, zero for new
//    Gaussians.
// The thresholds are formed in double on the host from the FP32 config and
// rounded to FP32, so every decision is an FP32 comparison.
//
// Plan and apply are two calls because the caller allocates the new arrays
// from the counts the plan writes.  The plan classifies each Gaussian and
// counts the classes per 256-Gaussian block, one block scans the counts; the
// apply recomputes each Gaussian's rank inside its block from ballots, so
// every class stays in the original order, and copies the block's rows group
// by group with consecutive threads on consecutive floats.  All kernels are
// bound by HBM traffic.
#include <cmath>
#include <string>

#include "gs_internal.h"

namespace gs {

constexpr int kDensThreads = 256;
constexpr int kDensWaves = kDensThreads / kWave;
constexpr int kScanThreads = 1024;
enum : uint8_t { kKeep = 1, kClone = 2, kSplit = 4 };

struct DensHalf {
  float sx[GS_MAX_VIEWS], sy[GS_MAX_VIEWS];  // W/2, H/2 per view
};

struct DensCfg {
  float tau, log_split, logit_min, log_div;
};

struct DensWs {
  uint8_t* cls;
  int32_t* block_counts;  // [nb][3]
  int32_t* block_offs;    // [nb][3]
  int32_t* totals;        // [3]
  size_t bytes;
};

static DensWs dens_ws(void* base, int64_t n) {
  const int64_t nb = (n + kDensThreads - 1) / kDensThreads;
  char* p = static_cast<char*>(base);
  DensWs w{};
  size_t off = 0;
  w.cls = reinterpret_cast<uint8_t*>(p + off);
  off += align256((size_t)n);
  w.block_counts = reinterpret_cast<int32_t*>(p + off);
  off += align256((size_t)nb * 3 * sizeof(int32_t));
  w.block_offs = reinterpret_cast<int32_t*>(p + off);
  off += align256((size_t)nb * 3 * sizeof(int32_t));
  w.totals = reinterpret_cast<int32_t*>(p + off);
  off += align256(3 * sizeof(int32_t));
  w.bytes = off;
  return w;
}

__global__ __launch_bounds__(kDensThreads) void k_density_accumulate(int64_t n, int n_views, DensHalf h,
                                                                       const int32_t* __restrict__ tiles,
                                                                       const float* __restrict__ grad2d,
                                                                       const float* __restrict__ abs2d,
                                                                       float* __restrict__ gacc,
                                                                       float* __restrict__ aacc,
                                                                       int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * kDensThreads + threadIdx.x;
  if (i >= n) return;
  float G = 0.0f, A = 0.0f;
  int c = 0;
#pragma unroll 4
  for (int v = 0; v < n_views; ++v) {
    const int64_t row = (int64_t)v * n + i;
    if (tiles[row] <= 0) continue;
    const float gx = h.sx[v] * grad2d[row * GS_GRAD2D_FLOATS], gy = h.sy[v] * grad2d[row * GS_GRAD2D_FLOATS + 1];
    const float ax = h.sx[v] * abs2d[row * 2], ay = h.sy[v] * abs2d[row * 2 + 1];
    G += sqrtf(fmaf(gx, gx, gy * gy));
    A += sqrtf(fmaf(ax, ax, ay * ay));
    ++c;
  }
  if (c > 0) {
    gacc[i] += G;
    aacc[i] += A;
    cnt[i] += c;
  }
}

// The class of Gaussian i (0 for i >= n).
__device__ inline uint8_t density_class(int64_t i, int64_t n, const float* __restrict__ log_scales,
                                        const float* __restrict__ logits, const float* __restrict__ aacc,
                                        const int32_t* __restrict__ cnt, const DensCfg& k) {
  if (i >= n) return 0;
  const int c = cnt[i];
  const bool sel = c > 0 && aacc[i] >= k.tau * (float)c;
  const float ls = fmaxf(fmaxf(log_scales[3 * i], log_scales[3 * i + 1]), log_scales[3 * i + 2]);
  const bool large = ls > k.log_split;
  const bool pruned = logits[i] < k.logit_min;
  if (pruned) return 0;
  if (!sel) return kKeep;
  return large ? kSplit : (uint8_t)(kKeep | kClone);
}

// Per class, this thread's rank among the block's members of the class, and the block's counts.
struct BlockRanks {
  int rank[3];
  int total[3];
};
__device__ inline BlockRanks block_ranks(uint8_t cls) {
  __shared__ int s_w[3][kDensWaves];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  unsigned long long m[3];
  m[0] = __ballot((cls & kKeep) != 0);
  m[1] = __ballot((cls & kClone) != 0);
  m[2] = __ballot((cls & kSplit) != 0);
  if (lane == 0)
    for (int k = 0; k < 3; ++k) s_w[k][w] = __popcll(m[k]);
  __syncthreads();
  BlockRanks r;
  for (int k = 0; k < 3; ++k) {
    int before = 0, tot = 0;
    for (int u = 0; u < kDensWaves; ++u) {
      before += u < w ? s_w[k][u] : 0;
      tot += s_w[k][u];
    }
    r.rank[k] = before + __popcll(m[k] & below);
    r.total[k] = tot;
  }
  return r;
}

__global__ __launch_bounds__(kDensThreads) void k_density_classify(int64_t n, const float* __restrict__ log_scales,
                                                                     const float* __restrict__ logits,
                                                                     const float* __restrict__ aacc,
                                                                     const int32_t* __restrict__ cnt, DensCfg k,
                                                                     uint8_t* __restrict__ cls,
                                                                     int32_t* __restrict__ block_counts) {
  const int64_t i = (int64_t)blockIdx.x * kDensThreads + threadIdx.x;
  const uint8_t c = density_class(i, n, log_scales, logits, aacc, cnt, k);
  if (i < n) cls[i] = c;
  const BlockRanks r = block_ranks(c);
  if (threadIdx.x < 3)
    block_counts[(int64_t)blockIdx.x * 3 + threadIdx.x] =
        threadIdx.x == 0 ? r.total[0] : (threadIdx.x == 1 ? r.total[1] : r.total[2]);
}

// One block: exclusive offsets of every block per class, and the class totals.
__global__ __launch_bounds__(kScanThreads) void k_density_scan(int64_t nb, const int32_t* __restrict__ block_counts,
                                                                int32_t* __restrict__ block_offs,
                                                                int32_t* __restrict__ totals,
                                                                int32_t* __restrict__ d_counts) {
  __shared__ int s_sum[kScanThreads];
  const int t = threadIdx.x;
  const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = (int64_t)t * per, b1 = b0 + per < nb ? b0 + per : nb;
  for (int k = 0; k < 3; ++k) {
    int local = 0;
    for (int64_t b = b0; b < b1; ++b) local += block_counts[b * 3 + k];
    s_sum[t] = local;
    __syncthreads();
    // inclusive scan of the per-thread sums (Hillis-Steele)
    for (int o = 1; o < kScanThreads; o <<= 1) {
      const int x = t >= o ? s_sum[t - o] : 0;
      __syncthreads();
      s_sum[t] += x;
      __syncthreads();
    }
    int run = s_sum[t] - local;
    for (int64_t b = b0; b < b1; ++b) {
      block_offs[b * 3 + k] = run;
      run += block_counts[b * 3 + k];
    }
    if (t == kScanThreads - 1) totals[k] = d_counts[k] = s_sum[t];
    __syncthreads();
  }
}

struct DensRows {
  const float* p[6];   // means, log_scales, quats, logits, sh_dc, sh_rest (source)
  const float* m[6];   // first moments
  const float* v[6];   // second moments
  float* op[6];        // destination parameters
  float* om[6];
  float* ov[6];
};

// Destinations of a block's rows, -1 where a row does not go: kept, clone, first and second child.
struct DensDst {
  int64_t keep[kDensThreads], clone[kDensThreads], child1[kDensThreads], child2[kDensThreads];
};

// One parameter group's rows of the block (W floats per Gaussian), copied cooperatively: consecutive
// threads take consecutive floats of the block's source rows, so the loads are coalesced, and as
// every class keeps the source order, consecutive rows of a class land on consecutive destination
// rows, so the stores are too.  New Gaussians get zero moments; CHILD copies the parameter into the
// split children (the means and log-scales of a child are computed, not copied).
template <int W, bool CHILD>
__device__ inline void scatter_group(const float* __restrict__ src, const float* __restrict__ sm,
                                     const float* __restrict__ sv, float* __restrict__ dp, float* __restrict__ dm,
                                     float* __restrict__ dv, int64_t i0, int rows, const DensDst& d) {
  if (W == 0) return;
  for (int f = threadIdx.x; f < rows * W; f += kDensThreads) {
    const int r = f / W, col = f - r * W;
    const int64_t jk = d.keep[r], jc = d.clone[r], j1 = d.child1[r], j2 = d.child2[r];
    if ((jk & jc & j1 & j2) < 0) continue;  // all -1: a pruned or split-only row with nothing to copy
    const int64_t si = (i0 + r) * W + col;
    if (jk >= 0) {
      dp[jk * W + col] = src[si];
      dm[jk * W + col] = sm[si];
      dv[jk * W + col] = sv[si];
    }
    if (jc >= 0) {
      dp[jc * W + col] = src[si];
      dm[jc * W + col] = 0.0f;
      dv[jc * W + col] = 0.0f;
    }
    if (j1 >= 0) {
      if (CHILD) dp[j1 * W + col] = src[si];
      dm[j1 * W + col] = 0.0f;
      dv[j1 * W + col] = 0.0f;
    }
    if (j2 >= 0) {
      if (CHILD) dp[j2 * W + col] = src[si];
      dm[j2 * W + col] = 0.0f;
      dv[j2 * W + col] = 0.0f;
    }
  }
}

template <int D>
__global__ __launch_bounds__(kDensThreads) void k_density_scatter(int64_t n, DensRows r, DensCfg k,
                                                                    const uint8_t* __restrict__ cls,
                                                                    const int32_t* __restrict__ block_offs,
                                                                    const int32_t* __restrict__ totals,
                                                                    const float* __restrict__ eps, int64_t n_eps,
                                                                    int64_t n_out) {
  constexpr int REST = 3 * ((D + 1) * (D + 1) - 1);
  __shared__ DensDst d;
  const int64_t i0 = (int64_t)blockIdx.x * kDensThreads, i = i0 + threadIdx.x;
  const int rows = (int)(n - i0 < kDensThreads ? n - i0 : kDensThreads);
  const uint8_t c = i < n ? cls[i] : (uint8_t)0;
  const BlockRanks br = block_ranks(c);
  const int64_t K = totals[0], C = totals[1], S = totals[2];
  const int32_t* off = block_offs + (int64_t)blockIdx.x * 3;
  const int64_t q = off[2] + br.rank[2];  // this row's split rank
  const bool has_eps = (q * 2 + 2) * 3 <= n_eps;
  const int64_t jk = (c & kKeep) ? off[0] + br.rank[0] : -1;
  const int64_t jc = (c & kClone) ? K + off[1] + br.rank[1] : -1;
  const int64_t j1 = (c & kSplit) && has_eps ? K + C + q : -1;
  const int64_t j2 = (c & kSplit) && has_eps ? K + C + S + q : -1;
  d.keep[threadIdx.x] = jk < n_out ? jk : -1;
  d.clone[threadIdx.x] = jc < n_out ? jc : -1;
  d.child1[threadIdx.x] = j1 < n_out ? j1 : -1;
  d.child2[threadIdx.x] = j2 < n_out ? j2 : -1;
  __syncthreads();
  scatter_group<3, false>(r.p[0], r.m[0], r.v[0], r.op[0], r.om[0], r.ov[0], i0, rows, d);
  scatter_group<3, false>(r.p[1], r.m[1], r.v[1], r.op[1], r.om[1], r.ov[1], i0, rows, d);
  scatter_group<4, true>(r.p[2], r.m[2], r.v[2], r.op[2], r.om[2], r.ov[2], i0, rows, d);
  scatter_group<1, true>(r.p[3], r.m[3], r.v[3], r.op[3], r.om[3], r.ov[3], i0, rows, d);
  scatter_group<3, true>(r.p[4], r.m[4], r.v[4], r.op[4], r.om[4], r.ov[4], i0, rows, d);
  scatter_group<REST, true>(r.p[5], r.m[5], r.v[5], r.op[5], r.om[5], r.ov[5], i0, rows, d);
  // the split children's means and log-scales
  const int64_t js[2] = {d.child1[threadIdx.x], d.child2[threadIdx.x]};
  if (js[0] < 0 && js[1] < 0) return;
  // rotation of the normalised quaternion (w, x, y, z) and the scales
  const float qw = r.p[2][4 * i], qx = r.p[2][4 * i + 1], qy = r.p[2][4 * i + 2], qz = r.p[2][4 * i + 3];
  const float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float w_ = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  const float R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w_ * z),     2 * (x * z + w_ * y),
                      2 * (x * y + w_ * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w_ * x),
                      2 * (x * z - w_ * y),     2 * (y * z + w_ * x),     1 - 2 * (x * x + y * y)};
  float s[3];
  for (int t = 0; t < 3; ++t) s[t] = expf(r.p[1][3 * i + t]);
  for (int child = 0; child < 2; ++child) {
    const int64_t j = js[child];
    if (j < 0) continue;
    const int64_t e = (q * 2 + child) * 3;
    float lv[3];
    for (int t = 0; t < 3; ++t) lv[t] = s[t] * eps[e + t];
    for (int t = 0; t < 3; ++t)
      r.op[0][3 * j + t] = r.p[0][3 * i + t] + fmaf(R[3 * t], lv[0], fmaf(R[3 * t + 1], lv[1], R[3 * t + 2] * lv[2]));
    for (int t = 0; t < 3; ++t) r.op[1][3 * j + t] = r.p[1][3 * i + t] - k.log_div;
  }
}

static DensCfg dens_cfg(const gs_density_config* c) {
  DensCfg k;
  k.tau = c->grad_threshold;
  k.log_split = (float)std::log((double)c->percent_dense * (double)c->extent);
  k.logit_min = (float)std::log((double)c->min_opacity / (1.0 - (double)c->min_opacity));
  k.log_div = (float)std::log((double)c->split_scale_div);
  return k;
}

static gs_status validate_density_cfg(const gs_density_config* c) {
  if (!c) return fail(GS_ERR_INVALID_VALUE, "cfg is NULL");
  if (!(c->grad_threshold >= 0.0f) || !std::isfinite(c->grad_threshold))
    return fail(GS_ERR_INVALID_VALUE, "grad_threshold must be finite and >= 0");
  if (!(c->percent_dense > 0.0f) || !(c->extent > 0.0f) || !std::isfinite(c->percent_dense * c->extent))
    return fail(GS_ERR_INVALID_VALUE, "percent_dense and extent must be finite and > 0");
  if (!(c->min_opacity > 0.0f && c->min_opacity < 1.0f))
    return fail(GS_ERR_INVALID_VALUE, "min_opacity must be in (0, 1)");
  if (!(c->split_scale_div > 0.0f) || !std::isfinite(c->split_scale_div))
    return fail(GS_ERR_INVALID_VALUE, "split_scale_div must be finite and > 0");
  return GS_OK;
}

static gs_status validate_stats(const gs_density_stats* s) {
  if (!s || !s->grad_accum || !s->abs_accum || !s->count) return fail(GS_ERR_INVALID_VALUE, "a statistics array is NULL");
  return GS_OK;
}

static gs_status rows_of(const gs_params* p, const char* what, const float* out[6]) {
  gs_status s;
  if ((s = validate_params(p)) != GS_OK) return fail(s, std::string(what) + ": " + gs_last_error());
  out[0] = p->means;
  out[1] = p->log_scales;
  out[2] = p->quats;
  out[3] = p->opacity_logits;
  out[4] = p->sh_dc;
  out[5] = p->sh_rest;
  return GS_OK;
}

static gs_status rows_out(const gs_grads* g, int D, const char* what, float* out[6]) {
  if (!g || !g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh_dc || (D > 0 && !g->sh_rest))
    return fail(GS_ERR_INVALID_VALUE, std::string(what) + ": an array is NULL");
  out[0] = g->means;
  out[1] = g->log_scales;
  out[2] = g->quats;
  out[3] = g->opacity_logits;
  out[4] = g->sh_dc;
  out[5] = g->sh_rest;
  return GS_OK;
}

}  // namespace gs

extern "C" void gs_default_density_config(gs_density_config* cfg) {
  if (!cfg) return;
  cfg->grad_threshold = 0.0002f;
  cfg->percent_dense = 0.01f;
  cfg->min_opacity = 0.005f;
  cfg->split_scale_div = 1.6f;
  cfg->extent = 1.0f;
}

extern "C" gs_status gs_scene_extent(const gs_camera* cams, int32_t n_views, float* extent) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if (!extent) return fail(GS_ERR_INVALID_VALUE, "extent is NULL");
  double c[GS_MAX_VIEWS][3], mean[3] = {0, 0, 0};
  for (int v = 0; v < n_views; ++v)
    for (int d = 0; d < 3; ++d) {
      // centre = -R^T t
      c[v][d] = -((double)cams[v].R[d] * cams[v].t[0] + (double)cams[v].R[3 + d] * cams[v].t[1] +
                  (double)cams[v].R[6 + d] * cams[v].t[2]);
      mean[d] += c[v][d] / n_views;
    }
  double r = 0.0;
  for (int v = 0; v < n_views; ++v) {
    const double dx = c[v][0] - mean[0], dy = c[v][1] - mean[1], dz = c[v][2] - mean[2];
    r = std::fmax(r, std::sqrt(dx * dx + dy * dy + dz * dz));
  }
  *extent = (float)(1.1 * r);
  return GS_OK;
}

extern "C" gs_status gs_density_accumulate(const gs_projected* proj, int64_t n, const gs_camera* cams,
                                           int32_t n_views, const float* grad2d, const float* abs_grad2d,
                                           const gs_density_stats* stats, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if (n < 1 || n > (int64_t(1) << 31)) return fail(GS_ERR_INVALID_VALUE, "n must be in [1, 2^31]");
  if (!proj || !proj->tiles_touched) return fail(GS_ERR_INVALID_VALUE, "proj->tiles_touched is NULL");
  if (!grad2d || !abs_grad2d) return fail(GS_ERR_INVALID_VALUE, "grad2d and abs_grad2d are required");
  if ((s = validate_stats(stats)) != GS_OK) return s;
  DensHalf h{};
  for (int v = 0; v < n_views; ++v) {
    h.sx[v] = 0.5f * (float)cams[v].width;
    h.sy[v] = 0.5f * (float)cams[v].height;
  }
  const unsigned nb = (unsigned)((n + kDensThreads - 1) / kDensThreads);
  hipLaunchKernelGGL(k_density_accumulate, dim3(nb), dim3(kDensThreads), 0, as_stream(stream), n, (int)n_views, h,
                     proj->tiles_touched, grad2d, abs_grad2d, stats->grad_accum, stats->abs_accum, stats->count);
  return check_launch("density statistics");
}

extern "C" gs_status gs_density_workspace_size(int64_t n, size_t* bytes) {
  using namespace gs;
  if (n < 1 || n > (int64_t(1) << 31)) return fail(GS_ERR_INVALID_VALUE, "n must be in [1, 2^31]");
  if (!bytes) return fail(GS_ERR_INVALID_VALUE, "bytes is NULL");
  *bytes = dens_ws(nullptr, n).bytes;
  return GS_OK;
}

extern "C" gs_status gs_density_plan(const gs_params* params, const gs_density_stats* stats,
                                     const gs_density_config* cfg, int32_t* d_counts, void* workspace,
                                     size_t workspace_bytes, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_params(params)) != GS_OK) return s;
  if ((s = validate_stats(stats)) != GS_OK) return s;
  if ((s = validate_density_cfg(cfg)) != GS_OK) return s;
  if (!d_counts) return fail(GS_ERR_INVALID_VALUE, "d_counts is NULL");
  const int64_t n = params->n;
  const DensWs w = dens_ws(workspace, n);
  if (!workspace || workspace_bytes < w.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(w.bytes) + " bytes");
  const DensCfg k = dens_cfg(cfg);
  const int64_t nb = (n + kDensThreads - 1) / kDensThreads;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_density_classify, dim3((unsigned)nb), dim3(kDensThreads), 0, st, n, params->log_scales,
                     params->opacity_logits, stats->abs_accum, stats->count, k, w.cls, w.block_counts);
  hipLaunchKernelGGL(k_density_scan, dim3(1), dim3(kScanThreads), 0, st, nb, w.block_counts, w.block_offs, w.totals,
                     d_counts);
  return check_launch("density plan");
}

extern "C" gs_status gs_density_apply(const gs_params* params, const gs_params* exp_avg, const gs_params* exp_avg_sq,
                                      const gs_density_config* cfg, const float* eps, int64_t n_eps, int64_t n_out,
                                      const gs_grads* out_params, const gs_grads* out_exp_avg,
                                      const gs_grads* out_exp_avg_sq, const void* workspace, size_t workspace_bytes,
                                      void* stream) {
  using namespace gs;
  gs_status s;
  DensRows r{};
  if ((s = rows_of(params, "params", r.p)) != GS_OK) return s;
  if ((s = rows_of(exp_avg, "exp_avg", r.m)) != GS_OK) return s;
  if ((s = rows_of(exp_avg_sq, "exp_avg_sq", r.v)) != GS_OK) return s;
  if ((s = validate_density_cfg(cfg)) != GS_OK) return s;
  const int64_t n = params->n;
  const int D = params->sh_degree;
  if (exp_avg->n != n || exp_avg_sq->n != n || exp_avg->sh_degree != D || exp_avg_sq->sh_degree != D)
    return fail(GS_ERR_INVALID_VALUE, "the moments must have the parameters' n and sh_degree");
  if (n_out < 0 || n_out > 3 * n) return fail(GS_ERR_INVALID_VALUE, "n_out must be in [0, 3 n]");
  if (n_eps < 0 || (n_eps > 0 && !eps)) return fail(GS_ERR_INVALID_VALUE, "eps is NULL with n_eps > 0");
  if (n_out > 0) {
    if ((s = rows_out(out_params, D, "out_params", r.op)) != GS_OK) return s;
    if ((s = rows_out(out_exp_avg, D, "out_exp_avg", r.om)) != GS_OK) return s;
    if ((s = rows_out(out_exp_avg_sq, D, "out_exp_avg_sq", r.ov)) != GS_OK) return s;
  }
  const DensWs w = dens_ws(const_cast<void*>(workspace), n);
  if (!workspace || workspace_bytes < w.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(w.bytes) + " bytes");
  if (n_out == 0) return GS_OK;
  const DensCfg k = dens_cfg(cfg);
  const int64_t nb = (n + kDensThreads - 1) / kDensThreads;
#define GS_SCATTER(DD)                                                                                         \
  hipLaunchKernelGGL(k_density_scatter<DD>, dim3((unsigned)nb), dim3(kDensThreads), 0, as_stream(stream), n, r, k, \
                     w.cls, w.block_offs, w.totals, eps, n_eps, n_out)
  switch (D) {
    case 0: GS_SCATTER(0); break;
    case 1: GS_SCATTER(1); break;
    case 2: GS_SCATTER(2); break;
    default: GS_SCATTER(3); break;
  }
#undef GS_SCATTER
  return check_launch("density apply");
}
