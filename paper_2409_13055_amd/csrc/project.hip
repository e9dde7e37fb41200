// Projection of the Gaussian set onto the keyframe image planes and its
// backward pass (Sec. II, first stage of the rasteriser; Gaussian
// parameterisation of Sec. III-B).
//
// One thread per Gaussian loops over every view of the call, so the 236 bytes
// of parameters of an SH-3 Gaussian are read from HBM once per call however
// many keyframes are rendered, and the records of view v are written as
// contiguous 48-byte rows (coalesced across the wavefront).
#include <cmath>
#include <cstring>

#include "gs_internal.h"

namespace gs {

struct ProjectArgs {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* logits;
  const float* sh_dc;
  const float* sh_rest;
  int64_t n;
  int32_t n_views;
  int32_t tile;
  float near_plane, eps2d, radius_sigmas, alpha_min;
};

struct GradPtrs {
  float* means;
  float* log_scales;
  float* quats;
  float* logits;
  float* sh_dc;
  float* sh_rest;
};

// Real spherical harmonics up to degree 3 (Condon-Shortley phase, order
// l, m = -l..l) at a unit direction.
__device__ inline void sh_basis(int D, float x, float y, float z, float* Y) {
  Y[0] = 0.28209479177387814f;
  if (D < 1) return;
  Y[1] = -0.4886025119029199f * y;
  Y[2] = 0.4886025119029199f * z;
  Y[3] = -0.4886025119029199f * x;
  if (D < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = 1.0925484305920792f * x * y;
  Y[5] = -1.0925484305920792f * y * z;
  Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
  Y[7] = -1.0925484305920792f * x * z;
  Y[8] = 0.5462742152960396f * (xx - yy);
  if (D < 3) return;
  Y[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
  Y[10] = 2.890611442640554f * x * y * z;
  Y[11] = -0.4570457994644658f * y * (4.0f * zz - xx - yy);
  Y[12] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -0.4570457994644658f * x * (4.0f * zz - xx - yy);
  Y[14] = 1.445305721320277f * z * (xx - yy);
  Y[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
}

// sum_k a_k grad(Y_k) of the polynomial forms above.
__device__ inline void sh_grad_dot(int D, float x, float y, float z, const float* a, float& gx, float& gy,
                                   float& gz) {
  gx = gy = gz = 0.0f;
  if (D < 1) return;
  const float c1 = 0.4886025119029199f;
  gy -= c1 * a[1];
  gz += c1 * a[2];
  gx -= c1 * a[3];
  if (D < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float c2a = 1.0925484305920792f, c2b = 0.31539156525252005f, c2c = 0.5462742152960396f;
  gx += c2a * y * a[4];
  gy += c2a * x * a[4];
  gy -= c2a * z * a[5];
  gz -= c2a * y * a[5];
  gx -= 2.0f * c2b * x * a[6];
  gy -= 2.0f * c2b * y * a[6];
  gz += 4.0f * c2b * z * a[6];
  gx -= c2a * z * a[7];
  gz -= c2a * x * a[7];
  gx += 2.0f * c2c * x * a[8];
  gy -= 2.0f * c2c * y * a[8];
  if (D < 3) return;
  const float k0 = -0.5900435899266435f, k1 = 2.890611442640554f, k2 = -0.4570457994644658f,
              k3 = 0.3731763325901154f, k5 = 1.445305721320277f;
  gx += k0 * 6.0f * x * y * a[9];
  gy += k0 * (3.0f * xx - 3.0f * yy) * a[9];
  gx += k1 * y * z * a[10];
  gy += k1 * x * z * a[10];
  gz += k1 * x * y * a[10];
  gx += k2 * (-2.0f * x * y) * a[11];
  gy += k2 * (4.0f * zz - xx - 3.0f * yy) * a[11];
  gz += k2 * 8.0f * y * z * a[11];
  gx += k3 * (-6.0f * x * z) * a[12];
  gy += k3 * (-6.0f * y * z) * a[12];
  gz += k3 * (6.0f * zz - 3.0f * xx - 3.0f * yy) * a[12];
  gx += k2 * (4.0f * zz - 3.0f * xx - yy) * a[13];
  gy += k2 * (-2.0f * x * y) * a[13];
  gz += k2 * 8.0f * x * z * a[13];
  gx += k5 * 2.0f * x * z * a[14];
  gy -= k5 * 2.0f * y * z * a[14];
  gz += k5 * (xx - yy) * a[14];
  gx += k0 * (3.0f * xx - 3.0f * yy) * a[15];
  gy += k0 * (-6.0f * x * y) * a[15];
}

// Geometry runs in double precision.  Both projection kernels are bound by
// HBM traffic (parameters in, records or gradients out), and gfx950 issues
// FP64 vector FMAs at the same rate as unpacked FP32 ones, so the wider type
// costs little time; it keeps the conic and the covariance chain rule accurate
// for very elongated or very large splats, where FP32 loses digits to
// cancellation (det of the 2D covariance, -Q G Q).  Colours stay FP32.
using real = double;

// View-independent part of a Gaussian: normalised quaternion, rotation,
// scales and the 3D covariance Sigma = (R S)(R S)^T.
struct Gauss3D {
  real m[3];
  real q[4];
  real qnorm;
  real R[9];
  real s[3];
  real M[9];    // R diag(s)
  real Sig[6];  // xx xy xz yy yz zz
  bool ok;
};

__device__ inline void load_gauss(const ProjectArgs& a, int64_t i, Gauss3D& g) {
  g.m[0] = a.means[3 * i];
  g.m[1] = a.means[3 * i + 1];
  g.m[2] = a.means[3 * i + 2];
  const float4 qf = *reinterpret_cast<const float4*>(a.quats + 4 * i);
  const real qw = qf.x, qx = qf.y, qy = qf.z, qz = qf.w;
  const real qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
  g.ok = qn2 > 0.0;
  g.qnorm = sqrt(qn2);
  const real inv = g.ok ? 1.0 / g.qnorm : 0.0;
  const real w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  g.q[0] = w; g.q[1] = x; g.q[2] = y; g.q[3] = z;
  g.R[0] = 1 - 2 * (y * y + z * z); g.R[1] = 2 * (x * y - w * z);     g.R[2] = 2 * (x * z + w * y);
  g.R[3] = 2 * (x * y + w * z);     g.R[4] = 1 - 2 * (x * x + z * z); g.R[5] = 2 * (y * z - w * x);
  g.R[6] = 2 * (x * z - w * y);     g.R[7] = 2 * (y * z + w * x);     g.R[8] = 1 - 2 * (x * x + y * y);
  for (int k = 0; k < 3; ++k) g.s[k] = exp((real)a.log_scales[3 * i + k]);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) g.M[3 * r + c] = g.R[3 * r + c] * g.s[c];
  const real* M = g.M;
  g.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  g.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  g.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  g.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  g.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  g.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
}

// What the per-view projection needs: the mean and the 3D covariance.
struct GaussCov {
  real m[3];
  real Sig[6];
  bool ok;
};

__device__ inline void load_cov(const ProjectArgs& a, int64_t i, GaussCov& c) {
  Gauss3D g;
  load_gauss(a, i, g);
  for (int k = 0; k < 3; ++k) c.m[k] = g.m[k];
  for (int k = 0; k < 6; ++k) c.Sig[k] = g.Sig[k];
  c.ok = g.ok;
}

// Per-view projection: camera point, guarded Jacobian J, T = J W, dilated
// 2D covariance, its inverse (conic) and the image-plane mean.
struct Proj2D {
  real t[3];
  real txc, tyc;
  real cvx, cvy;   // clamp value of x/z, y/z when the guard is active
  bool clx, cly;
  real T[6];
  real a, b, c;    // dilated covariance
  real ca, cb, cc; // conic
  real mx, my;
};

__device__ inline bool project_view(const GaussCov& g, const CamF& cam, real near_plane, real eps2d, Proj2D& p) {
  const real W[9] = {cam.R[0], cam.R[1], cam.R[2], cam.R[3], cam.R[4], cam.R[5], cam.R[6], cam.R[7], cam.R[8]};
  const real fx = cam.fx, fy = cam.fy, limx = cam.limx, limy = cam.limy;
  for (int r = 0; r < 3; ++r)
    p.t[r] = W[3 * r] * g.m[0] + W[3 * r + 1] * g.m[1] + W[3 * r + 2] * g.m[2] + (real)cam.t[r];
  if (!(p.t[2] > near_plane)) return false;
  const real iz = 1.0 / p.t[2];
  const real ux = p.t[0] * iz, uy = p.t[1] * iz;
  p.clx = ux < -limx || ux > limx;
  p.cly = uy < -limy || uy > limy;
  p.cvx = fmin(fmax(ux, -limx), limx);
  p.cvy = fmin(fmax(uy, -limy), limy);
  p.txc = p.clx ? p.cvx * p.t[2] : p.t[0];
  p.tyc = p.cly ? p.cvy * p.t[2] : p.t[1];
  const real j00 = fx * iz, j02 = -fx * p.txc * iz * iz;
  const real j11 = fy * iz, j12 = -fy * p.tyc * iz * iz;
  for (int c = 0; c < 3; ++c) {
    p.T[c] = j00 * W[c] + j02 * W[6 + c];
    p.T[3 + c] = j11 * W[3 + c] + j12 * W[6 + c];
  }
  const real* S = g.Sig;
  const real* T = p.T;
  // (T Sigma) rows
  const real u0 = T[0] * S[0] + T[1] * S[1] + T[2] * S[2];
  const real u1 = T[0] * S[1] + T[1] * S[3] + T[2] * S[4];
  const real u2 = T[0] * S[2] + T[1] * S[4] + T[2] * S[5];
  const real w0 = T[3] * S[0] + T[4] * S[1] + T[5] * S[2];
  const real w1 = T[3] * S[1] + T[4] * S[3] + T[5] * S[4];
  const real w2 = T[3] * S[2] + T[4] * S[4] + T[5] * S[5];
  p.a = u0 * T[0] + u1 * T[1] + u2 * T[2] + eps2d;
  p.b = u0 * T[3] + u1 * T[4] + u2 * T[5];
  p.c = w0 * T[3] + w1 * T[4] + w2 * T[5] + eps2d;
  const real det = p.a * p.c - p.b * p.b;
  if (!(det > 0.0)) return false;
  const real idet = 1.0 / det;
  p.ca = p.c * idet;
  p.cb = -p.b * idet;
  p.cc = p.a * idet;
  p.mx = fx * p.t[0] * iz + (real)cam.cx - 0.5;
  p.my = fy * p.t[1] * iz + (real)cam.cy - 0.5;
  return true;
}

// Unit viewing direction from the camera centre to the mean (d) and
// 1/|mean - centre| (il).  Shared by the projection and its backward, whose
// colour-clamp decisions must agree.  The offset is formed in FP64 (a camera
// far from the scene keeps its digits) and normalised in FP32: the direction
// only feeds the FP32 colour evaluation and the colour's share of the mean
// gradient.
__device__ inline void view_dir(const GaussCov& g, const CamF& cam, float d[3], float& il) {
  const float dx = (float)(g.m[0] - (real)cam.centre[0]), dy = (float)(g.m[1] - (real)cam.centre[1]),
              dz = (float)(g.m[2] - (real)cam.centre[2]);
  il = rsqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
  d[0] = dx * il;
  d[1] = dy * il;
  d[2] = dz * il;
}

// One colour channel before the clamp at 0: 1/2 + sum_k sh_k Y_k, in one fixed
// FMA order (coef(k, c) returns coefficient k of channel c).
template <int K, class Coef>
__device__ __forceinline__ float sh_channel(const Coef& coef, const float* Y, int c) {
  float s = 0.5f;
#pragma unroll
  for (int k = 0; k < K; ++k) s = fmaf(coef(k, c), Y[k], s);
  return s;
}

// Besides the records, each wavefront (64 consecutive Gaussians) lists its
// visible pairs of every view in ascending i, at their ballot prefix within
// the segment of (view, wavefront), with the segment's count.
template <int D>
__global__ __launch_bounds__(256) void k_project(ProjectArgs a, CamTable cams, float* __restrict__ rec,
                                                 int32_t* __restrict__ tiles_touched, uint4* __restrict__ vis,
                                                 uint32_t* __restrict__ vis_count) {
  constexpr int K = (D + 1) * (D + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t n_seg = (a.n + 63) >> 6;
  GaussCov g;
  load_cov(a, i, g);
  float sh[K][3];
  sh[0][0] = a.sh_dc[3 * i];
  sh[0][1] = a.sh_dc[3 * i + 1];
  sh[0][2] = a.sh_dc[3 * i + 2];
#pragma unroll
  for (int k = 1; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[k][c] = a.sh_rest[(i * (K - 1) + (k - 1)) * 3 + c];
  const real o64 = 1.0 / (1.0 + exp(-(real)a.logits[i]));
  const float op = (float)o64;
  // Tile rect half-extents: the axis-aligned box of the region where opacity * exp(-q/2) can reach
  // alpha' = alpha_min (1 - 1e-3), cut to the radius_sigmas square, plus one pixel (the rect covers
  // every pixel within extent - 1 of the mean); opacity <= alpha' never blends and is culled.
  const real alpha_p = (real)a.alpha_min * (1.0 - 1e-3);
  const bool opaque_enough = o64 > alpha_p;
  const real thr = opaque_enough ? 2.0 * log(o64 / alpha_p) : 0.0;
  const int B = a.tile;
#pragma unroll 1
  for (int v = 0; v < a.n_views; ++v) {
    const CamF& cam = cams.c[v];
    Proj2D p;
    // a Gaussian too transparent to ever blend is culled before its projection is computed
    bool ok = g.ok && opaque_enough && project_view(g, cam, a.near_plane, a.eps2d, p);
    int packed = 0, tiles = 0;
    int x0 = 0, y0 = 0, x1 = 0, y1 = 0;
    float rgb[3] = {0.f, 0.f, 0.f};
    uint32_t flags = 0;
    const float fmx = ok ? (float)p.mx : 0.f, fmy = ok ? (float)p.my : 0.f;
    if (ok) {
      // the integer extents from FP32 square roots of FP64 arguments: they differ from FP64 roots only
      // where a root lies within a few 1e-7 of an integer (the FP32 rounding of the argument and of
      // the root), a boundary case of the extents either way
      const real mid = 0.5 * (p.a + p.c);
      const float lam = (float)mid + sqrtf((float)fmax(mid * mid - (p.a * p.c - p.b * p.b), 0.0));
      const float r = fminf(ceilf(a.radius_sigmas * sqrtf(lam)), (float)kMaxExtent);
      const int rx = (int)fminf(r, ceilf(sqrtf((float)(thr * p.a))) + 1.0f);
      const int ry = (int)fminf(r, ceilf(sqrtf((float)(thr * p.c))) + 1.0f);
      const int TX = (cam.W + B - 1) / B, TY = (cam.H + B - 1) / B;
      tile_rect(fmx, fmy, rx, ry, B, TX, TY, x0, y0, x1, y1);
      tiles = (x1 - x0) * (y1 - y0);
      if (tiles <= 0) {
        ok = false;
        tiles = 0;
      } else {
        packed = rx | (ry << 16);
      }
    }
    if (ok) {
      float d[3], il;
      view_dir(g, cam, d, il);
      float Y[16];
      sh_basis(D, d[0], d[1], d[2], Y);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float s = sh_channel<K>([&](int k, int ch) { return sh[k][ch]; }, Y, c);
        if (s < 0.0f) {
          flags |= 1u << c;
          s = 0.0f;
        }
        rgb[c] = s;
      }
      if (p.clx) flags |= 1u << 3;
      if (p.cly) flags |= 1u << 4;
    }
    const int64_t row = (int64_t)v * a.n + i;
    // only a visible pair's record is written: every later stage reads records through the tile
    // lists, and most pairs of a multi-view batch are culled, so their 48 bytes would be write
    // traffic nobody reads
    if (ok) {
      float4* out = reinterpret_cast<float4*>(rec + row * GS_REC_FLOATS);
      out[0] = make_float4(fmx, fmy, (float)p.ca, (float)p.cb);
      out[1] = make_float4((float)p.cc, op, rgb[0], rgb[1]);
      out[2] = make_float4(rgb[2], (float)p.t[2], __int_as_float(packed), __uint_as_float(flags));
    }
    tiles_touched[row] = tiles;
    const uint64_t bal = __ballot(ok);
    const int64_t seg = (int64_t)v * n_seg + (i >> 6);
    if (ok)
      vis[seg * 64 + __popcll(bal & below)] = make_uint4((uint32_t)x0 | ((uint32_t)x1 << 16),
                                                         (uint32_t)y0 | ((uint32_t)y1 << 16), (uint32_t)row,
                                                         __float_as_uint((float)p.t[2]));
    if (lane == 0) vis_count[seg] = (uint32_t)__popcll(bal);
  }
}

// Adam state of the fused projection backward: per parameter group (means,
// log_scales, quats, opacity logits, sh_dc, sh_rest) the parameters (updated
// in place), first and second moments and learning rate.
constexpr int kParamGroups = 6;
struct AdamPtrs {
  float* p[kParamGroups];
  float* m[kParamGroups];
  float* v[kParamGroups];
  float lr[kParamGroups];
  AdamCoef c;
  const int32_t* d_step;
};

// Backward of the projection: one thread per Gaussian sums the image-space
// gradients of all its views, accumulating the view-independent d/dSigma
// once, then chains to log-scales and the (unnormalised) quaternion.  The
// raw-parameter gradient of a Gaussian some view sees is added into `gp`.
// With ADAM the gradients of the block's Gaussians (0 where no view sees one)
// are instead staged in LDS in the parameter arrays' own layout and used at
// once for the Adam step of every parameter, the same update the standalone
// step applies, the block streaming each group's contiguous range of p, m and
// v as float4 with consecutive lanes on consecutive elements.
// With STATS the thread also adds its Gaussian's density-control statistics
// of the iteration (the norms of the view-space and homodirectional
// gradients in normalised device units, and the count of views whose tiles
// it touches), exactly as the standalone statistics kernel does, so grad2d is
// read once.
struct DensAcc {
  const float* abs2d;
  float* gacc;
  float* aacc;
  int32_t* cnt;
};
constexpr int kBwdThreads = 256;
template <int D, bool ADAM, bool STATS>
__global__ __launch_bounds__(kBwdThreads) void k_project_bwd(ProjectArgs a, CamTable cams,
                                                             const int32_t* __restrict__ tiles,
                                                             const float* __restrict__ grad2d, GradPtrs gp,
                                                             AdamPtrs ap, DensAcc da) {
  constexpr int K = (D + 1) * (D + 1);
  constexpr int NPAR = 11 + 3 * K;  // raw floats per Gaussian
  __shared__ __align__(16) float s_g[ADAM ? kBwdThreads * NPAR : 1];
  const int64_t i = (int64_t)blockIdx.x * kBwdThreads + threadIdx.x;
  const bool valid = i < a.n;
  if (!ADAM && !valid) return;
  // the raw-parameter gradient of Gaussian i (all 0 when no view sees it)
  float gmean[3] = {0.f, 0.f, 0.f}, glsc[3] = {0.f, 0.f, 0.f}, gquat[4] = {0.f, 0.f, 0.f, 0.f}, glogit = 0.f;
  float gsh[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.0f;
  GaussCov g;
  g.ok = false;
  if (valid) load_cov(a, i, g);
  if (g.ok) {
    // SH coefficients are re-read per view (cache hits) instead of held in
    // registers across the view loop.
    const float* shd = a.sh_dc + 3 * i;
    const float* shr = a.sh_rest + i * (K - 1) * 3;
    real gm[3] = {0, 0, 0};
    real gS[6] = {0, 0, 0, 0, 0, 0};
    real gop = 0;
    bool any = false;
    float sG = 0.0f, sA = 0.0f;  // STATS: this iteration's norms summed over views
    int sC = 0;
    // the views that see the Gaussian (tiles_touched > 0), eight loads in flight at a time
    uint32_t seen = 0;
#pragma unroll 1
    for (int v0 = 0; v0 < a.n_views; v0 += 8) {
      int32_t t[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) t[k] = tiles[(int64_t)min(v0 + k, a.n_views - 1) * a.n + i];
#pragma unroll
      for (int k = 0; k < 8; ++k) seen |= (v0 + k < a.n_views && t[k] != 0) ? 1u << (v0 + k) : 0u;
    }
    // (the view index stays the same in every lane, so camera data are scalar loads)
#pragma unroll 1
    for (int v = 0; v < a.n_views; ++v) {
      const bool sees = (seen >> v) & 1u;
      if (__ballot(sees) == 0ull) continue;  // no lane's Gaussian is seen by this view
      if (!sees) continue;                   // culled: no image-space gradient
      const int64_t row = (int64_t)v * a.n + i;
      real g2[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) g2[k] = grad2d[row * 9 + k];
      const CamF& cam = cams.c[v];
      if (STATS) {
        const float hx = 0.5f * (float)cam.W, hy = 0.5f * (float)cam.H;
        const float gx = hx * (float)g2[0], gy = hy * (float)g2[1];
        const float ax = hx * da.abs2d[row * 2], ay = hy * da.abs2d[row * 2 + 1];
        sG += sqrtf(fmaf(gx, gx, gy * gy));
        sA += sqrtf(fmaf(ax, ax, ay * ay));
        ++sC;
      }
      Proj2D p;
      if (!project_view(g, cam, a.near_plane, a.eps2d, p)) continue;
      any = true;
      // conic -> covariance: dL/dcov = -Q GQ Q
      const real A = p.ca, Bq = p.cb, C = p.cc;
      const real ga = g2[2], gb = 0.5 * g2[3], gc = g2[4];
      const real q00 = A * ga + Bq * gb, q01 = A * gb + Bq * gc;
      const real q10 = Bq * ga + C * gb, q11 = Bq * gb + C * gc;
      const real G00 = -(q00 * A + q01 * Bq);
      const real G01 = -(q00 * Bq + q01 * C);
      const real G11 = -(q10 * Bq + q11 * C);
      // cov = T Sigma T^T (dilation is additive): dL/dSigma = T^T G T, dL/dT = 2 G T Sigma
      const real* T = p.T;
      real u[3], w[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        u[k] = G00 * T[k] + G01 * T[3 + k];
        w[k] = G01 * T[k] + G11 * T[3 + k];
      }
      gS[0] += T[0] * u[0] + T[3] * w[0];
      gS[1] += T[0] * u[1] + T[3] * w[1];
      gS[2] += T[0] * u[2] + T[3] * w[2];
      gS[3] += T[1] * u[1] + T[4] * w[1];
      gS[4] += T[1] * u[2] + T[4] * w[2];
      gS[5] += T[2] * u[2] + T[5] * w[2];
      const real* S = g.Sig;
      const real GT0[3] = {2 * (u[0] * S[0] + u[1] * S[1] + u[2] * S[2]), 2 * (u[0] * S[1] + u[1] * S[3] + u[2] * S[4]),
                           2 * (u[0] * S[2] + u[1] * S[4] + u[2] * S[5])};
      const real GT1[3] = {2 * (w[0] * S[0] + w[1] * S[1] + w[2] * S[2]), 2 * (w[0] * S[1] + w[1] * S[3] + w[2] * S[4]),
                           2 * (w[0] * S[2] + w[1] * S[4] + w[2] * S[5])};
      const real Wc[9] = {cam.R[0], cam.R[1], cam.R[2], cam.R[3], cam.R[4], cam.R[5], cam.R[6], cam.R[7], cam.R[8]};
      const real fx = cam.fx, fy = cam.fy;
      // dL/dJ = dL/dT W^T (entries J00, J02, J11, J12)
      const real gj00 = GT0[0] * Wc[0] + GT0[1] * Wc[1] + GT0[2] * Wc[2];
      const real gj02 = GT0[0] * Wc[6] + GT0[1] * Wc[7] + GT0[2] * Wc[8];
      const real gj11 = GT1[0] * Wc[3] + GT1[1] * Wc[4] + GT1[2] * Wc[5];
      const real gj12 = GT1[0] * Wc[6] + GT1[1] * Wc[7] + GT1[2] * Wc[8];
      const real tz = p.t[2], iz = 1.0 / tz, iz2 = iz * iz, iz3 = iz2 * iz;
      real gt0 = 0, gt1 = 0, gt2 = 0;
      gt2 += gj00 * (-fx * iz2) + gj11 * (-fy * iz2);
      gt0 += p.clx ? 0.0 : gj02 * (-fx * iz2);
      gt2 += gj02 * (-fx * iz2 * (p.clx ? p.cvx : 0.0) + 2.0 * fx * p.txc * iz3);
      gt1 += p.cly ? 0.0 : gj12 * (-fy * iz2);
      gt2 += gj12 * (-fy * iz2 * (p.cly ? p.cvy : 0.0) + 2.0 * fy * p.tyc * iz3);
      // image-plane mean
      gt0 += g2[0] * fx * iz;
      gt1 += g2[1] * fy * iz;
      gt2 -= (g2[0] * fx * p.t[0] + g2[1] * fy * p.t[1]) * iz2;
      gm[0] += Wc[0] * gt0 + Wc[3] * gt1 + Wc[6] * gt2;
      gm[1] += Wc[1] * gt0 + Wc[4] * gt1 + Wc[7] * gt2;
      gm[2] += Wc[2] * gt0 + Wc[5] * gt1 + Wc[8] * gt2;
      gop += g2[5];
      // colour -> SH coefficients and the viewing direction; a channel clamped at 0 in the
      // projection (same arithmetic as there) passes no gradient
      float d[3], il;
      view_dir(g, cam, d, il);
      const float dx = d[0], dy = d[1], dz = d[2];
      float Y[16], acoef[16];
      sh_basis(D, dx, dy, dz, Y);
      const auto coef = [&](int k, int ch) { return (k == 0 ? shd : shr + (k - 1) * 3)[ch]; };
      const float wr = sh_channel<K>(coef, Y, 0) < 0.0f ? 0.f : (float)g2[6];
      const float wg = sh_channel<K>(coef, Y, 1) < 0.0f ? 0.f : (float)g2[7];
      const float wb = sh_channel<K>(coef, Y, 2) < 0.0f ? 0.f : (float)g2[8];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        gsh[k][0] += wr * Y[k];
        gsh[k][1] += wg * Y[k];
        gsh[k][2] += wb * Y[k];
        const float* c3 = k == 0 ? shd : shr + (k - 1) * 3;
        acoef[k] = wr * c3[0] + wg * c3[1] + wb * c3[2];
      }
      if (D > 0) {
        float gdx, gdy, gdz;
        sh_grad_dot(D, dx, dy, dz, acoef, gdx, gdy, gdz);
        const float dd = gdx * dx + gdy * dy + gdz * dz;
        gm[0] += (gdx - dx * dd) * il;
        gm[1] += (gdy - dy * dd) * il;
        gm[2] += (gdz - dz * dd) * il;
      }
    }
    if (any) {
      Gauss3D gf;  // rotation, scales and M = R diag(s), recomputed after the view loop
      load_gauss(a, i, gf);
      // Sigma = M M^T, M = R diag(s): dL/dM = 2 gS M
      const real GSm[9] = {gS[0], gS[1], gS[2], gS[1], gS[3], gS[4], gS[2], gS[4], gS[5]};
      real GM[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          GM[3 * r + c] = 2 * (GSm[3 * r] * gf.M[c] + GSm[3 * r + 1] * gf.M[3 + c] + GSm[3 * r + 2] * gf.M[6 + c]);
      real gls[3], GR[9];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const real gsv = GM[c] * gf.R[c] + GM[3 + c] * gf.R[3 + c] + GM[6 + c] * gf.R[6 + c];
        gls[c] = gsv * gf.s[c];
        GR[c] = GM[c] * gf.s[c];
        GR[3 + c] = GM[3 + c] * gf.s[c];
        GR[6 + c] = GM[6 + c] * gf.s[c];
      }
      const real w = gf.q[0], x = gf.q[1], y = gf.q[2], z = gf.q[3];
      // d R / d(w,x,y,z) contracted with GR
      const real gw = 2 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
      const real gx = 2 * (y * GR[1] + z * GR[2] + y * GR[3] - 2 * x * GR[4] - w * GR[5] + z * GR[6] + w * GR[7] -
                           2 * x * GR[8]);
      const real gy = 2 * (-2 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7] -
                           2 * y * GR[8]);
      const real gz = 2 * (-2 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2 * z * GR[4] + y * GR[5] +
                           x * GR[6] + y * GR[7]);
      const real dotq = w * gw + x * gx + y * gy + z * gz;
      const real iq = 1.0 / gf.qnorm;
      const real op = 1.0 / (1.0 + exp(-(real)a.logits[i]));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gmean[c] = (float)gm[c];
        glsc[c] = (float)gls[c];
      }
      gquat[0] = (float)((gw - w * dotq) * iq);
      gquat[1] = (float)((gx - x * dotq) * iq);
      gquat[2] = (float)((gy - y * dotq) * iq);
      gquat[3] = (float)((gz - z * dotq) * iq);
      glogit = (float)(gop * op * (1.0 - op));
      if (!ADAM) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          gp.means[3 * i + c] += gmean[c];
          gp.log_scales[3 * i + c] += glsc[c];
        }
        float4* gq = reinterpret_cast<float4*>(gp.quats + 4 * i);
        float4 qv = *gq;
        qv.x += gquat[0];
        qv.y += gquat[1];
        qv.z += gquat[2];
        qv.w += gquat[3];
        *gq = qv;
        gp.logits[i] += glogit;
#pragma unroll
        for (int c = 0; c < 3; ++c) gp.sh_dc[3 * i + c] += gsh[0][c];
#pragma unroll
        for (int k = 1; k < K; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) gp.sh_rest[(i * (K - 1) + (k - 1)) * 3 + c] += gsh[k][c];
      }
    }  // any
    if (STATS && sC > 0) {
      da.gacc[i] += sG;
      da.aacc[i] += sA;
      da.cnt[i] += sC;
    }
  }  // g.ok
  if (!ADAM) return;
  // group g's block of gradients sits at s_g[T * off_g + t * width_g + c], as in the group's array
  constexpr int T = kBwdThreads;
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s_g[0 * T + t * 3 + c] = gmean[c];
    s_g[3 * T + t * 3 + c] = glsc[c];
    s_g[11 * T + t * 3 + c] = gsh[0][c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) s_g[6 * T + t * 4 + c] = gquat[c];
  s_g[10 * T + t] = glogit;
#pragma unroll
  for (int k = 1; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) s_g[14 * T + t * 3 * (K - 1) + (k - 1) * 3 + c] = gsh[k][c];
  __shared__ float s_k[2];
  if (t == 0) adam_bias_factors(ap.c, *ap.d_step, s_k[0], s_k[1]);
  __syncthreads();
  const float k1 = s_k[0], k2 = s_k[1];
  const int64_t i0 = (int64_t)blockIdx.x * T;
  const int nb = (int)min<int64_t>(T, a.n - i0);
  const int width[kParamGroups] = {3, 3, 4, 1, 3, 3 * (K - 1)};
  const int off[kParamGroups] = {0, 3, 6, 10, 11, 14};
  // Each group's range of the block as float4 (it starts 16-byte aligned: i0 is a multiple of 256),
  // four chunks per thread at a time with all their loads in flight before any update or store;
  // the last block's remainder one by one.
#pragma unroll
  for (int grp = 0; grp < kParamGroups; ++grp) {
    const int w = width[grp];
    if (w == 0) continue;
    const float* G = s_g + off[grp] * T;
    float* __restrict__ P = ap.p[grp] + i0 * w;
    float* __restrict__ M = ap.m[grp] + i0 * w;
    float* __restrict__ V = ap.v[grp] + i0 * w;
    const float step_size = ap.lr[grp] * k1;
    const int cnt = nb * w, n4 = (((reinterpret_cast<uintptr_t>(P) | reinterpret_cast<uintptr_t>(M) |
                                    reinterpret_cast<uintptr_t>(V)) & 15) == 0) ? cnt / 4 : 0;
    constexpr int U = 4;
    for (int q0 = t; q0 < n4; q0 += U * T) {
      float4 pv[U], mv[U], vv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = min(q0 + u * T, n4 - 1);  // clamped: every load in bounds, the extra ones unused
        pv[u] = reinterpret_cast<const float4*>(P)[q];
        mv[u] = reinterpret_cast<const float4*>(M)[q];
        vv[u] = reinterpret_cast<const float4*>(V)[q];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * T;
        if (q >= n4) break;
        const float4 gv = reinterpret_cast<const float4*>(G)[q];
        adam_update(pv[u].x, gv.x, mv[u].x, vv[u].x, ap.c, step_size, k2);
        adam_update(pv[u].y, gv.y, mv[u].y, vv[u].y, ap.c, step_size, k2);
        adam_update(pv[u].z, gv.z, mv[u].z, vv[u].z, ap.c, step_size, k2);
        adam_update(pv[u].w, gv.w, mv[u].w, vv[u].w, ap.c, step_size, k2);
        reinterpret_cast<float4*>(P)[q] = pv[u];
        reinterpret_cast<float4*>(M)[q] = mv[u];
        reinterpret_cast<float4*>(V)[q] = vv[u];
      }
    }
    for (int e = 4 * n4 + t; e < cnt; e += T) {
      float pv = P[e], mv = M[e], vv = V[e];
      adam_update(pv, G[e], mv, vv, ap.c, step_size, k2);
      P[e] = pv;
      M[e] = mv;
      V[e] = vv;
    }
  }
}

static ProjectArgs make_args(const gs_params* p, int32_t n_views, const gs_options* o) {
  ProjectArgs a;
  a.means = p->means;
  a.log_scales = p->log_scales;
  a.quats = p->quats;
  a.logits = p->opacity_logits;
  a.sh_dc = p->sh_dc;
  a.sh_rest = p->sh_rest;
  a.n = p->n;
  a.n_views = n_views;
  a.tile = o->tile_size;
  a.near_plane = o->near_plane;
  a.eps2d = o->eps2d;
  a.radius_sigmas = o->radius_sigmas;
  a.alpha_min = o->alpha_min;
  return a;
}

gs_status validate_params(const gs_params* p) {
  if (!p) return fail(GS_ERR_INVALID_VALUE, "params is NULL");
  if (p->n < 1 || p->n > (int64_t(1) << 31)) return fail(GS_ERR_INVALID_VALUE, "params->n must be in [1, 2^31]");
  if (p->sh_degree < 0 || p->sh_degree > GS_MAX_SH_DEGREE)
    return fail(GS_ERR_INVALID_VALUE, "sh_degree must be in [0, 3]");
  if (!p->means || !p->log_scales || !p->quats || !p->opacity_logits || !p->sh_dc)
    return fail(GS_ERR_INVALID_VALUE, "a parameter pointer is NULL");
  if (p->sh_degree > 0 && !p->sh_rest) return fail(GS_ERR_INVALID_VALUE, "sh_rest is NULL with sh_degree > 0");
  if (reinterpret_cast<uintptr_t>(p->quats) % 16 != 0)
    return fail(GS_ERR_INVALID_VALUE, "quats must be 16-byte aligned");
  return GS_OK;
}

template <bool ADAM, bool STATS = false>
static void launch_project_bwd_kernel(const gs_params* params, const ProjectArgs& a, const CamTable& ct,
                                      const int32_t* tiles, const float* grad2d, const GradPtrs& gp,
                                      const AdamPtrs& ap, hipStream_t stream, const DensAcc& da = DensAcc{}) {
  const int bs = kBwdThreads;
  const dim3 grid((unsigned)((params->n + bs - 1) / bs));
#define GS_PBWD(DD) \
  hipLaunchKernelGGL((k_project_bwd<DD, ADAM, STATS>), grid, dim3(bs), 0, stream, a, ct, tiles, grad2d, gp, ap, da)
  switch (params->sh_degree) {
    case 0: GS_PBWD(0); break;
    case 1: GS_PBWD(1); break;
    case 2: GS_PBWD(2); break;
    default: GS_PBWD(3); break;
  }
#undef GS_PBWD
}

gs_status launch_project_bwd(const gs_params* params, const gs_camera* cams, int32_t n_views, const gs_options* opts,
                             const int32_t* tiles, const float* grad2d, const gs_grads* grads, hipStream_t stream) {
  const ProjectArgs a = make_args(params, n_views, opts);
  const CamTable ct = make_cam_table(cams, n_views, opts);
  GradPtrs gp{grads->means, grads->log_scales, grads->quats, grads->opacity_logits, grads->sh_dc, grads->sh_rest};
  launch_project_bwd_kernel<false>(params, a, ct, tiles, grad2d, gp, AdamPtrs{}, stream);
  return check_launch("projection backward");
}

}  // namespace gs

namespace gs {
static gs_status project_bwd_adam(const gs_params* params, const gs_projected* proj, const gs_camera* cams,
                                  int32_t n_views, const gs_options* opts, const float* grad2d,
                                  const gs_adam_group* groups, double beta1, double beta2, double eps, int32_t* d_step,
                                  const float* abs_grad2d, const gs_density_stats* stats, void* stream) {
  gs_status s;
  if ((s = validate_params(params)) != GS_OK) return s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if (!proj || !proj->tiles_touched) return fail(GS_ERR_INVALID_VALUE, "proj->tiles_touched is NULL");
  if (!grad2d) return fail(GS_ERR_INVALID_VALUE, "grad2d is NULL");
  if ((s = validate_adam_hyper(beta1, beta2, eps, d_step)) != GS_OK) return s;
  if (!groups) return fail(GS_ERR_INVALID_VALUE, "groups is NULL");
  const int K = (params->sh_degree + 1) * (params->sh_degree + 1);
  const float* owned[kParamGroups] = {params->means, params->log_scales, params->quats, params->opacity_logits,
                                      params->sh_dc, params->sh_rest};
  const int64_t width[kParamGroups] = {3, 3, 4, 1, 3, 3 * (K - 1)};
  AdamPtrs ap{};
  for (int k = 0; k < kParamGroups; ++k) {
    const gs_adam_group& gr = groups[k];
    const std::string which = "group " + std::to_string(k);
    if (gr.numel != params->n * width[k]) return fail(GS_ERR_INVALID_VALUE, which + ": numel != n * width");
    if (gr.numel > 0 && (gr.param != owned[k] || !gr.exp_avg || !gr.exp_avg_sq))
      return fail(GS_ERR_INVALID_VALUE, which + ": param must be the params array, moments non-NULL");
    if (!std::isfinite(gr.lr)) return fail(GS_ERR_INVALID_VALUE, which + ": lr not finite");
    ap.p[k] = gr.param;
    ap.m[k] = gr.exp_avg;
    ap.v[k] = gr.exp_avg_sq;
    ap.lr[k] = gr.lr;
  }
  ap.c = make_adam_coef(beta1, beta2, eps);
  ap.d_step = d_step;
  const ProjectArgs a = make_args(params, n_views, opts);
  const CamTable ct = make_cam_table(cams, n_views, opts);
  hipStream_t st = as_stream(stream);
  if (stats)
    launch_project_bwd_kernel<true, true>(params, a, ct, proj->tiles_touched, grad2d, GradPtrs{}, ap, st,
                                          DensAcc{abs_grad2d, stats->grad_accum, stats->abs_accum, stats->count});
  else
    launch_project_bwd_kernel<true>(params, a, ct, proj->tiles_touched, grad2d, GradPtrs{}, ap, st);
  launch_step_increment(d_step, st);
  return check_launch("projection backward + adam");
}
}  // namespace gs

extern "C" gs_status gs_project_bwd_adam(const gs_params* params, const gs_projected* proj, const gs_camera* cams,
                                         int32_t n_views, const gs_options* opts, const float* grad2d,
                                         const gs_adam_group* groups, double beta1, double beta2, double eps,
                                         int32_t* d_step, void* stream) {
  return gs::project_bwd_adam(params, proj, cams, n_views, opts, grad2d, groups, beta1, beta2, eps, d_step, nullptr,
                              nullptr, stream);
}

extern "C" gs_status gs_project_bwd_adam_stats(const gs_params* params, const gs_projected* proj,
                                               const gs_camera* cams, int32_t n_views, const gs_options* opts,
                                               const float* grad2d, const gs_adam_group* groups, double beta1,
                                               double beta2, double eps, int32_t* d_step, const float* abs_grad2d,
                                               const gs_density_stats* stats, void* stream) {
  using namespace gs;
  if (!abs_grad2d) return fail(GS_ERR_INVALID_VALUE, "abs_grad2d is NULL");
  if (!stats || !stats->grad_accum || !stats->abs_accum || !stats->count)
    return fail(GS_ERR_INVALID_VALUE, "a statistics array is NULL");
  return project_bwd_adam(params, proj, cams, n_views, opts, grad2d, groups, beta1, beta2, eps, d_step, abs_grad2d,
                          stats, stream);
}

extern "C" gs_status gs_project(const gs_params* params, const gs_camera* cams, int32_t n_views,
                                const gs_options* opts, const gs_projected* out, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_params(params)) != GS_OK) return s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if (!out || !out->rec || !out->tiles_touched || !out->vis || !out->vis_count)
    return fail(GS_ERR_INVALID_VALUE, "out/rec/tiles_touched/vis/vis_count is NULL");
  if (reinterpret_cast<uintptr_t>(out->rec) % 16 != 0) return fail(GS_ERR_INVALID_VALUE, "rec must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(out->vis) % 16 != 0) return fail(GS_ERR_INVALID_VALUE, "vis must be 16-byte aligned");
  if ((int64_t)n_views * params->n >= (int64_t(1) << 32) - 1)
    return fail(GS_ERR_INVALID_VALUE, "n_views * n must be < 2^32 - 1");
  const ProjectArgs a = make_args(params, n_views, opts);
  const CamTable ct = make_cam_table(cams, n_views, opts);
  const int bs = 256;
  const dim3 grid((unsigned)((params->n + bs - 1) / bs));
  hipStream_t st = as_stream(stream);
  uint4* vis = reinterpret_cast<uint4*>(out->vis);
  uint32_t* vc = out->vis_count;
  switch (params->sh_degree) {
    case 0: hipLaunchKernelGGL(k_project<0>, grid, dim3(bs), 0, st, a, ct, out->rec, out->tiles_touched, vis, vc); break;
    case 1: hipLaunchKernelGGL(k_project<1>, grid, dim3(bs), 0, st, a, ct, out->rec, out->tiles_touched, vis, vc); break;
    case 2: hipLaunchKernelGGL(k_project<2>, grid, dim3(bs), 0, st, a, ct, out->rec, out->tiles_touched, vis, vc); break;
    default: hipLaunchKernelGGL(k_project<3>, grid, dim3(bs), 0, st, a, ct, out->rec, out->tiles_touched, vis, vc); break;
  }
  return check_launch("projection");
}
