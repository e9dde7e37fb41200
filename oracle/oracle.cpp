/*
 * FP64 CPU oracle for the tile-based differentiable 3D Gaussian splatting
 * rasteriser of the dense-reconstruction module (Sec. III-B) and its
 * gradient.  Rendering takes the three stages of Sec. II: a perspective
 * projection of each Gaussian to a 2D splat, a depth order per screen tile,
 * and front-to-back compositing per pixel.
 * The gradient is that of the L1 term of the photometric loss, eq. (2), with
 * respect to the five per-Gaussian quantities of Sec. III-B (opacity,
 * rotation, location, scale, colour).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may load this
 * library: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the
 * HIP implementation.
 *
 * The paper gives no formulas for the rasteriser (it defers to the original
 * 3DGS rasteriser, Sec. III-B).  The mathematics written out here is the
 * elliptical-weighted-average splatting model with the following readings,
 * each a field of the options struct so both implementations see one value:
 *   camera   pinhole, p_c = R p_w + t, x right / y down / z forward;
 *   pixels   pixel (i,j) is sampled at the integer point (i,j) of index
 *            coordinates, i.e. the image-plane mean is (u - 1/2, v - 1/2);
 *   near     a Gaussian with camera depth <= near_plane is culled;
 *   guard    the Jacobian uses x/z clamped to +-guard*(W/2)/fx (same for y);
 *   dilation eps2d * I is added to the 2D covariance (opacity unchanged);
 *   radius   r = ceil(radius_sigmas * sqrt(largest eigenvalue)), at most 32767;
 *   extents  the tile rect follows the axis-aligned box of the region where
 *            opacity * exp(-q/2) can reach alpha' = alpha_min (1 - 1e-3),
 *            cut to the r square: half-extents rx = min(r, ceil(sqrt(thr
 *            S_xx)) + 1), ry = min(r, ceil(sqrt(thr S_yy)) + 1), thr =
 *            2 ln(opacity / alpha'), S the dilated 2D covariance; opacity
 *            <= alpha' culls.  The rect formula below covers every pixel
 *            within extent - 1 of the mean (not always the last pixel before
 *            mean + extent), hence the + 1.  Every tile of the r square left
 *            out holds no pixel the blending would take, so the image is
 *            that of the r-square rects;
 *   rect     tiles [floor((m-rx)/B), floor((m+rx+B-1)/B)) in FP32 (same
 *            for y), clamped;
 *   alpha    min(alpha_max, o exp(power)); skipped below alpha_min;
 *   stop     a Gaussian that would take transmittance below t_min is not
 *            blended and ends the pixel;
 *   colour   real spherical harmonics (Condon-Shortley phase) plus 1/2,
 *            clamped at 0; degree 0 is the plain-RGB mode of Sec. III-B.
 *
 * Everything is double precision except the tile rectangle and the sort key,
 * which are defined on FP32 values (the key is the FP32 bit pattern of the
 * depth), because those are discrete decisions both sides must reproduce.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

struct OrCamera {
  double R[9];  // world -> camera rotation, row major
  double t[3];
  double fx, fy, cx, cy;
  int32_t width, height;
};

struct OrOptions {
  int32_t tile;
  int32_t reserved;
  double near_plane, eps2d, alpha_min, alpha_max, t_min, radius_sigmas, guard;
  double bg[3];
};

}  // extern "C"

namespace {

const double kPi = 3.14159265358979323846;

// Projected-record layout (doubles per (view, Gaussian)).
enum { R_MX = 0, R_MY, R_DEPTH, R_CA, R_CB, R_CC, R_OP, R_R, R_G, R_B, R_STRIDE };
// Per-(view, Gaussian) flag bits.
enum : uint32_t {
  F_CLAMP_R = 1u << 0, F_CLAMP_G = 1u << 1, F_CLAMP_B = 1u << 2,
  F_GUARD_X = 1u << 3, F_GUARD_Y = 1u << 4,
  F_CULL_NEAR = 1u << 8, F_CULL_DET = 1u << 9, F_CULL_RECT = 1u << 10, F_CULL_QUAT = 1u << 11,
  F_CULL_OPACITY = 1u << 12,
  F_NEAR_RADIUS = 1u << 16, F_NEAR_RECT = 1u << 17, F_NEAR_PLANE = 1u << 18,
};
// Per-pixel flag bits: a decision within a relative margin of its threshold.
enum : uint32_t { P_NEAR_ALPHA_MIN = 1u, P_NEAR_T_MIN = 2u, P_NEAR_ALPHA_MAX = 4u, P_NEAR_POWER0 = 8u };

inline int sh_count(int D) { return (D + 1) * (D + 1); }

// ---------------------------------------------------------------------------
// Real spherical harmonics up to degree 3, orthonormal on the unit sphere,
// Condon-Shortley phase, order (l, m = -l..l).  The constants are the
// normalisations sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 for
// m != 0) folded into the Cartesian polynomial of each function.
// ---------------------------------------------------------------------------
struct Sh {
  double c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e;
  Sh() {
    c0 = 0.5 * std::sqrt(1.0 / kPi);
    c1 = std::sqrt(3.0 / (4.0 * kPi));
    c2a = 0.5 * std::sqrt(15.0 / kPi);
    c2b = 0.25 * std::sqrt(5.0 / kPi);
    c2c = 0.25 * std::sqrt(15.0 / kPi);
    c3a = 0.25 * std::sqrt(35.0 / (2.0 * kPi));
    c3b = 0.5 * std::sqrt(105.0 / kPi);
    c3c = 0.25 * std::sqrt(21.0 / (2.0 * kPi));
    c3d = 0.25 * std::sqrt(7.0 / kPi);
    c3e = 0.25 * std::sqrt(105.0 / kPi);
  }
  // Y[k] at the unit vector d; G[k][3] = gradient of the polynomial form.
  void eval(int D, const double d[3], double* Y, double (*G)[3]) const {
    const double x = d[0], y = d[1], z = d[2];
    auto set = [&](int k, double v, double gx, double gy, double gz) {
      Y[k] = v;
      if (G) { G[k][0] = gx; G[k][1] = gy; G[k][2] = gz; }
    };
    set(0, c0, 0, 0, 0);
    if (D < 1) return;
    set(1, -c1 * y, 0, -c1, 0);
    set(2, c1 * z, 0, 0, c1);
    set(3, -c1 * x, -c1, 0, 0);
    if (D < 2) return;
    set(4, c2a * x * y, c2a * y, c2a * x, 0);
    set(5, -c2a * y * z, 0, -c2a * z, -c2a * y);
    set(6, c2b * (3 * z * z - 1), 0, 0, 6 * c2b * z);
    set(7, -c2a * x * z, -c2a * z, 0, -c2a * x);
    set(8, c2c * (x * x - y * y), 2 * c2c * x, -2 * c2c * y, 0);
    if (D < 3) return;
    set(9, -c3a * (3 * x * x * y - y * y * y), -c3a * 6 * x * y, -c3a * (3 * x * x - 3 * y * y), 0);
    set(10, c3b * x * y * z, c3b * y * z, c3b * x * z, c3b * x * y);
    set(11, -c3c * y * (5 * z * z - 1), 0, -c3c * (5 * z * z - 1), -c3c * 10 * y * z);
    set(12, c3d * (5 * z * z * z - 3 * z), 0, 0, c3d * (15 * z * z - 3));
    set(13, -c3c * x * (5 * z * z - 1), -c3c * (5 * z * z - 1), 0, -c3c * 10 * x * z);
    set(14, c3e * z * (x * x - y * y), 2 * c3e * x * z, -2 * c3e * y * z, c3e * (x * x - y * y));
    set(15, -c3a * (x * x * x - 3 * x * y * y), -c3a * (3 * x * x - 3 * y * y), c3a * 6 * x * y, 0);
  }
};
const Sh kSh;

// Rotation matrix of the unit quaternion (w,x,y,z) and its partial derivatives.
void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}
void quat_to_rot_grad(const double q[4], double dR[4][9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  const double dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  const double dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  const double dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  std::memcpy(dR[0], dw, sizeof dw);
  std::memcpy(dR[1], dx, sizeof dx);
  std::memcpy(dR[2], dy, sizeof dy);
  std::memcpy(dR[3], dz, sizeof dz);
}

inline bool near_integer(double v, double rel) {
  return std::fabs(v - std::nearbyint(v)) <= rel * std::max(1.0, std::fabs(v));
}

struct TileGrid {
  int tx, ty;
};
inline TileGrid grid_of(int W, int H, int B) { return {(W + B - 1) / B, (H + B - 1) / B}; }

// Tile rectangle [x0,x1) x [y0,y1) of a splat with half-extents (rx, ry),
// defined on FP32 values.
void tile_rect(float mx, float my, int rx, int ry, int B, TileGrid g, int rect[4]) {
  const float ex = (float)rx, ey = (float)ry, fb = (float)B, fb1 = (float)(B - 1);
  float x0 = std::floor((mx - ex) / fb), x1 = std::floor(((mx + ex) + fb1) / fb);
  float y0 = std::floor((my - ey) / fb), y1 = std::floor(((my + ey) + fb1) / fb);
  auto cl = [](float v, int hi) { return (int)std::min(std::max(v, 0.0f), (float)hi); };
  rect[0] = cl(x0, g.tx); rect[1] = cl(y0, g.ty); rect[2] = cl(x1, g.tx); rect[3] = cl(y1, g.ty);
}

inline uint32_t f32_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

// ---------------------------------------------------------------------------
// Projection of one Gaussian into one view, with the intermediates the
// backward pass needs.
// ---------------------------------------------------------------------------
struct ProjOut {
  double rec[R_STRIDE];
  int radius;   // r, 0 when culled
  int ext[2];   // (rx, ry), 0 when culled
  int rect[4];
  uint32_t flags;
  double cov[3];  // dilated 2D covariance (a, b, c)
};

struct GaussIn {
  const double* mean;
  const double* log_scale;
  const double* quat;
  double logit;
  const double* sh;  // [K][3]
};

void project_one(const GaussIn& gi, int D, const OrCamera& cam, const OrOptions& o, ProjOut& out) {
  std::memset(&out, 0, sizeof out);
  const double* Rc = cam.R;
  const double* m = gi.mean;
  double t[3];
  for (int r = 0; r < 3; ++r) t[r] = Rc[3 * r] * m[0] + Rc[3 * r + 1] * m[1] + Rc[3 * r + 2] * m[2] + cam.t[r];
  out.rec[R_DEPTH] = t[2];
  const double qn2 = gi.quat[0] * gi.quat[0] + gi.quat[1] * gi.quat[1] + gi.quat[2] * gi.quat[2] +
                     gi.quat[3] * gi.quat[3];
  if (std::fabs(t[2] - o.near_plane) <= 1e-6 * std::max(1.0, o.near_plane)) out.flags |= F_NEAR_PLANE;
  if (qn2 == 0.0) { out.flags |= F_CULL_QUAT; return; }
  if (t[2] <= o.near_plane) { out.flags |= F_CULL_NEAR; return; }

  // Image-plane mean in index coordinates.
  out.rec[R_MX] = cam.fx * t[0] / t[2] + cam.cx - 0.5;
  out.rec[R_MY] = cam.fy * t[1] / t[2] + cam.cy - 0.5;

  // 3D covariance Sigma = (R S)(R S)^T.
  const double qn = std::sqrt(qn2);
  const double q[4] = {gi.quat[0] / qn, gi.quat[1] / qn, gi.quat[2] / qn, gi.quat[3] / qn};
  double Rq[9];
  quat_to_rot(q, Rq);
  const double s[3] = {std::exp(gi.log_scale[0]), std::exp(gi.log_scale[1]), std::exp(gi.log_scale[2])};
  double M[9], Sig[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += M[3 * i + k] * M[3 * j + k];
      Sig[3 * i + j] = a;
    }

  // Affine approximation of the perspective map at t (with the frustum guard).
  const double limx = o.guard * 0.5 * cam.width / cam.fx, limy = o.guard * 0.5 * cam.height / cam.fy;
  double ux = t[0] / t[2], uy = t[1] / t[2];
  double txc = t[0], tyc = t[1];
  if (ux < -limx || ux > limx) { out.flags |= F_GUARD_X; ux = std::min(std::max(ux, -limx), limx); txc = ux * t[2]; }
  if (uy < -limy || uy > limy) { out.flags |= F_GUARD_Y; uy = std::min(std::max(uy, -limy), limy); tyc = uy * t[2]; }
  const double iz = 1.0 / t[2];
  const double J[6] = {cam.fx * iz, 0, -cam.fx * txc * iz * iz, 0, cam.fy * iz, -cam.fy * tyc * iz * iz};
  double T[6];  // J * Rc (2x3)
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) T[3 * i + j] = J[3 * i] * Rc[j] + J[3 * i + 1] * Rc[3 + j] + J[3 * i + 2] * Rc[6 + j];
  double TS[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) TS[3 * i + j] = T[3 * i] * Sig[j] + T[3 * i + 1] * Sig[3 + j] + T[3 * i + 2] * Sig[6 + j];
  double a = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2];
  double b = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
  double c = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5];
  a += o.eps2d;
  c += o.eps2d;
  out.cov[0] = a; out.cov[1] = b; out.cov[2] = c;
  const double det = a * c - b * b;
  if (!(det > 0)) { out.flags |= F_CULL_DET; return; }
  out.rec[R_CA] = c / det;
  out.rec[R_CB] = -b / det;
  out.rec[R_CC] = a / det;
  const double mid = 0.5 * (a + c);
  const double lam = mid + std::sqrt(std::max(mid * mid - det, 0.0));
  const double rr = o.radius_sigmas * std::sqrt(lam);
  out.radius = (int)std::min(std::ceil(rr), 32767.0);  // extents saturate at 32767 px
  if (near_integer(rr, 1e-5)) out.flags |= F_NEAR_RADIUS;

  // Opacity-aware half-extents of the tile rect (see the header).
  const double opacity = 1.0 / (1.0 + std::exp(-gi.logit));
  const double alpha_p = o.alpha_min * (1.0 - 1e-3);
  if (std::fabs(opacity / alpha_p - 1.0) <= 1e-9) out.flags |= F_NEAR_RADIUS;
  if (!(opacity > alpha_p)) {
    out.flags |= F_CULL_OPACITY;
    out.radius = 0;
    return;
  }
  const double thr = 2.0 * std::log(opacity / alpha_p);
  const double ex = std::sqrt(thr * a), ey = std::sqrt(thr * c);
  out.ext[0] = (int)std::min((double)out.radius, std::ceil(ex) + 1.0);
  out.ext[1] = (int)std::min((double)out.radius, std::ceil(ey) + 1.0);
  if (near_integer(ex, 1e-5) || near_integer(ey, 1e-5)) out.flags |= F_NEAR_RADIUS;

  const int B = o.tile;
  const TileGrid g = grid_of(cam.width, cam.height, B);
  tile_rect((float)out.rec[R_MX], (float)out.rec[R_MY], out.ext[0], out.ext[1], B, g, out.rect);
  {
    const double fx = out.ext[0], fy = out.ext[1];
    const double args[4] = {(out.rec[R_MX] - fx) / B, (out.rec[R_MX] + fx + B - 1) / B,
                            (out.rec[R_MY] - fy) / B, (out.rec[R_MY] + fy + B - 1) / B};
    for (double v : args)
      if (near_integer(v, 1e-5)) out.flags |= F_NEAR_RECT;
  }
  if (out.rect[2] <= out.rect[0] || out.rect[3] <= out.rect[1]) {
    out.flags |= F_CULL_RECT;
    out.radius = 0;
    out.ext[0] = out.ext[1] = 0;
    std::memset(out.rect, 0, sizeof out.rect);
    return;
  }

  // Colour from spherical harmonics at the viewing direction.
  const double cc[3] = {-(Rc[0] * cam.t[0] + Rc[3] * cam.t[1] + Rc[6] * cam.t[2]),
                        -(Rc[1] * cam.t[0] + Rc[4] * cam.t[1] + Rc[7] * cam.t[2]),
                        -(Rc[2] * cam.t[0] + Rc[5] * cam.t[1] + Rc[8] * cam.t[2])};
  double d[3] = {m[0] - cc[0], m[1] - cc[1], m[2] - cc[2]};
  const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  d[0] /= dn; d[1] /= dn; d[2] /= dn;
  double Y[16];
  kSh.eval(D, d, Y, nullptr);
  for (int ch = 0; ch < 3; ++ch) {
    double v = 0.5;
    for (int k = 0; k < sh_count(D); ++k) v += gi.sh[3 * k + ch] * Y[k];
    if (v < 0) { out.flags |= (F_CLAMP_R << ch); v = 0; }
    out.rec[R_R + ch] = v;
  }
  out.rec[R_OP] = opacity;
}

struct ViewInfo {
  OrCamera cam;
  TileGrid grid;
  int64_t tile_off;
  int64_t pix_off;
};

std::vector<ViewInfo> make_views(const OrCamera* cams, int nv, int B) {
  std::vector<ViewInfo> v(nv);
  int64_t to = 0, po = 0;
  for (int i = 0; i < nv; ++i) {
    v[i].cam = cams[i];
    v[i].grid = grid_of(cams[i].width, cams[i].height, B);
    v[i].tile_off = to;
    v[i].pix_off = po;
    to += (int64_t)v[i].grid.tx * v[i].grid.ty;
    po += (int64_t)cams[i].width * cams[i].height;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Front-to-back blending of one pixel over its tile's depth-ordered list.
// ---------------------------------------------------------------------------
struct Accepted {
  uint32_t id;   // v*N + i
  int k;         // position in the tile list
  double alpha, G, T, dx, dy;
  bool clamped;  // o*G exceeded alpha_max
};

// A decision of the blending at one list entry that lies within the FP32
// rounding bound of its threshold: `kind` is the P_NEAR_* bit of the test.
struct FlaggedDecision {
  int k;
  uint32_t kind;
};
constexpr int kMaxFlagged = 8;

struct PixelTrace {
  std::vector<Accepted> acc;
  double C[3];
  double T;
  int n_contrib;
  uint32_t flags;
  int stop_k;  // list position of the Gaussian that ended the pixel, or -1
  // the first kMaxFlagged near-threshold decisions in list order, and their number
  FlaggedDecision flagged[kMaxFlagged];
  int n_flagged;
  // smallest relative distance of an evaluated entry's alpha from alpha_min, and of
  // a blended or stopping entry's transmittance from t_min
  double margin_alpha, margin_t;
};

// The decision at list position flip.k of kind flip.kind is taken the other
// way (for the alternatives an FP32 evaluation may produce at a flagged
// decision); flip.k < 0 takes every decision as the definition says.
struct Flip {
  int k = -1;
  uint32_t kind = 0;
};

void trace_pixel(double px, double py, const uint32_t* list, int64_t len, const double* rec, const OrOptions& o,
                 bool keep, PixelTrace& tr, uint32_t ov_id = 0xffffffffu, const double* ov_row = nullptr,
                 Flip flip = Flip()) {
  tr.acc.clear();
  tr.C[0] = tr.C[1] = tr.C[2] = 0;
  tr.T = 1.0;
  tr.n_contrib = 0;
  tr.flags = 0;
  tr.stop_k = -1;
  tr.n_flagged = 0;
  tr.margin_alpha = tr.margin_t = INFINITY;
  auto flag = [&](int64_t k, uint32_t kind) {
    tr.flags |= kind;
    if (tr.n_flagged < kMaxFlagged) tr.flagged[tr.n_flagged] = {(int)k, kind};
    ++tr.n_flagged;
  };
  auto flipped = [&](int64_t k, uint32_t kind, bool decision) {
    return (k == flip.k && kind == flip.kind) ? !decision : decision;
  };
  // Relative uncertainty of an FP32 evaluation of T so far (for the flags).
  double t_rel = 0.0;
  const double u = std::ldexp(1.0, -24);  // FP32 unit roundoff
  for (int64_t k = 0; k < len; ++k) {
    const double* g = (list[k] == ov_id) ? ov_row : rec + (size_t)list[k] * R_STRIDE;
    const double dx = px - g[R_MX], dy = py - g[R_MY];
    const double power = -0.5 * (g[R_CA] * dx * dx + g[R_CC] * dy * dy) - g[R_CB] * dx * dy;
    // A decision counts as "near" its threshold when it lies within the
    // rounding error an FP32 evaluation of the same expression can make:
    // the quadratic form loses accuracy to cancellation in proportion to the
    // magnitude of its terms (elongated splats), plus exp and the products.
    const double terms = std::fabs(g[R_CA] * dx * dx) + std::fabs(g[R_CC] * dy * dy) + 2 * std::fabs(g[R_CB] * dx * dy);
    // the sign of the exponent: its absolute FP32 error is that of the quadratic form
    if (std::fabs(power) < 8 * u * terms) flag(k, P_NEAR_POWER0);
    if (flipped(k, P_NEAR_POWER0, power > 0)) continue;
    const double G = std::exp(power);
    const double oG = g[R_OP] * G;
    const double a_rel = 1e-5 + 8 * u * terms + 2 * u * std::fabs(power);
    if (std::fabs(oG - o.alpha_max) <= a_rel * o.alpha_max) flag(k, P_NEAR_ALPHA_MAX);
    const bool clamped = flipped(k, P_NEAR_ALPHA_MAX, oG > o.alpha_max);
    const double alpha = clamped ? o.alpha_max : oG;
    if (std::fabs(alpha - o.alpha_min) <= a_rel * o.alpha_min) flag(k, P_NEAR_ALPHA_MIN);
    tr.margin_alpha = std::min(tr.margin_alpha, std::fabs(alpha - o.alpha_min) / o.alpha_min);
    if (flipped(k, P_NEAR_ALPHA_MIN, alpha < o.alpha_min)) continue;
    const double nextT = tr.T * (1.0 - alpha);
    tr.margin_t = std::min(tr.margin_t, std::fabs(nextT - o.t_min) / o.t_min);
    const double step_rel = (clamped ? 0.0 : a_rel * alpha / (1.0 - alpha)) + 2 * u;
    if (std::fabs(nextT - o.t_min) <= (1e-4 + t_rel + step_rel) * o.t_min) flag(k, P_NEAR_T_MIN);
    t_rel += step_rel;
    if (flipped(k, P_NEAR_T_MIN, nextT < o.t_min)) { tr.stop_k = (int)k; break; }
    for (int ch = 0; ch < 3; ++ch) tr.C[ch] += g[R_R + ch] * alpha * tr.T;
    if (keep) tr.acc.push_back({list[k], (int)k, alpha, G, tr.T, dx, dy, clamped});
    tr.T = nextT;
    tr.n_contrib = (int)k + 1;
  }
}

// Backward of one pixel: adds d(loss)/d(record) of every blended Gaussian.
// Row layout: (mx, my, ca, cb, cc, opacity, r, g, b), then the magnitudes of
// this pixel's two mean components, |dL_pixel/dmx| and |dL_pixel/dmy|, whose
// sums over pixels are the homodirectional (AbsGS) view-space gradient, then
// for each of the nine terms the magnitude of the parts it is formed from
// (their sums over pixels scale the rounding error of any evaluation of the
// gradient): dL/dalpha = sum_c dl_c (col_c T - S_c / (1 - alpha)) is taken
// with |col_c| T + (|S_c| + C_c) / (1 - alpha), C the pixel's colour, because
// an evaluation that recovers the colour behind an entry by subtracting the
// colour in front of it from C carries an error relative to C, not to S.
constexpr int kRowW = 20;
void backward_pixel(const PixelTrace& tr, const double dl[3], const double* rec, const OrOptions& o,
                    double* rows /* [len][kRowW], indexed by list position */) {
  double S[3] = {tr.T * o.bg[0], tr.T * o.bg[1], tr.T * o.bg[2]};
  const double Cpix[3] = {tr.C[0] + S[0], tr.C[1] + S[1], tr.C[2] + S[2]};
  for (size_t a = tr.acc.size(); a-- > 0;) {
    const Accepted& e = tr.acc[a];
    const double* g = rec + (size_t)e.id * R_STRIDE;
    double* row = rows + (size_t)e.k * kRowW;
    double t[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double dl_dalpha = 0, dl_dalpha_mag = 0;
    for (int ch = 0; ch < 3; ++ch) {
      t[6 + ch] = dl[ch] * e.alpha * e.T;
      m[6 + ch] = std::fabs(t[6 + ch]);
      dl_dalpha += dl[ch] * (g[R_R + ch] * e.T - S[ch] / (1.0 - e.alpha));
      dl_dalpha_mag += std::fabs(dl[ch]) * (std::fabs(g[R_R + ch]) * e.T +
                                            (std::fabs(S[ch]) + std::fabs(Cpix[ch])) / (1.0 - e.alpha));
      S[ch] += g[R_R + ch] * e.alpha * e.T;
    }
    if (!e.clamped) {
      const double dl_dpower = dl_dalpha * e.alpha, mp = dl_dalpha_mag * e.alpha;
      const double geo[5] = {g[R_CA] * e.dx + g[R_CB] * e.dy, g[R_CB] * e.dx + g[R_CC] * e.dy, -0.5 * e.dx * e.dx,
                             -e.dx * e.dy, -0.5 * e.dy * e.dy};
      t[5] = dl_dalpha * e.G;
      m[5] = dl_dalpha_mag * e.G;
      for (int c = 0; c < 5; ++c) {
        t[c] = dl_dpower * geo[c];
        m[c] = mp * std::fabs(geo[c]);
      }
      row[9] += std::fabs(t[0]);
      row[10] += std::fabs(t[1]);
    }
    for (int c = 0; c < 9; ++c) {
      row[c] += t[c];
      row[11 + c] += m[c];
    }
  }
}

// Locate (view, local tile) of a global tile id.
inline int view_of_tile(const std::vector<ViewInfo>& views, int64_t gt) {
  int v = 0;
  while (v + 1 < (int)views.size() && views[v + 1].tile_off <= gt) ++v;
  return v;
}

// ---------------------------------------------------------------------------
// Backward of the projection for one Gaussian in one view: chain the 9 image-
// space gradients to the raw parameters (accumulated into the outputs).
// ---------------------------------------------------------------------------
void project_backward_one(const GaussIn& gi, int D, const OrCamera& cam, const OrOptions& o, const double g2[9],
                          double* gm, double* gls, double* gq, double* glogit, double* gsh) {
  ProjOut po;
  project_one(gi, D, cam, o, po);
  if (po.radius <= 0) return;
  const double* Rc = cam.R;
  const double* m = gi.mean;
  double t[3];
  for (int r = 0; r < 3; ++r) t[r] = Rc[3 * r] * m[0] + Rc[3 * r + 1] * m[1] + Rc[3 * r + 2] * m[2] + cam.t[r];
  const double qn2 = gi.quat[0] * gi.quat[0] + gi.quat[1] * gi.quat[1] + gi.quat[2] * gi.quat[2] +
                     gi.quat[3] * gi.quat[3];
  const double qn = std::sqrt(qn2);
  const double q[4] = {gi.quat[0] / qn, gi.quat[1] / qn, gi.quat[2] / qn, gi.quat[3] / qn};
  double Rq[9];
  quat_to_rot(q, Rq);
  const double s[3] = {std::exp(gi.log_scale[0]), std::exp(gi.log_scale[1]), std::exp(gi.log_scale[2])};
  double M[9], Sig[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += M[3 * i + k] * M[3 * j + k];
      Sig[3 * i + j] = a;
    }
  const double limx = o.guard * 0.5 * cam.width / cam.fx, limy = o.guard * 0.5 * cam.height / cam.fy;
  const double ux = t[0] / t[2], uy = t[1] / t[2];
  const bool clx = ux < -limx || ux > limx, cly = uy < -limy || uy > limy;
  const double cvx = clx ? std::min(std::max(ux, -limx), limx) : 0.0;
  const double cvy = cly ? std::min(std::max(uy, -limy), limy) : 0.0;
  const double txc = clx ? cvx * t[2] : t[0];
  const double tyc = cly ? cvy * t[2] : t[1];
  const double iz = 1.0 / t[2];
  const double J[6] = {cam.fx * iz, 0, -cam.fx * txc * iz * iz, 0, cam.fy * iz, -cam.fy * tyc * iz * iz};
  double T[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) T[3 * i + j] = J[3 * i] * Rc[j] + J[3 * i + 1] * Rc[3 + j] + J[3 * i + 2] * Rc[6 + j];

  // conic -> 2D covariance: dL/dcov = -Q G_Q Q with Q the conic matrix.
  const double A = po.rec[R_CA], Bc = po.rec[R_CB], C = po.rec[R_CC];
  const double GQ[4] = {g2[2], 0.5 * g2[3], 0.5 * g2[3], g2[4]};
  const double Q[4] = {A, Bc, Bc, C};
  double QG[4], Gc[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) QG[2 * i + j] = Q[2 * i] * GQ[j] + Q[2 * i + 1] * GQ[2 + j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) Gc[2 * i + j] = -(QG[2 * i] * Q[j] + QG[2 * i + 1] * Q[2 + j]);
  // cov = T Sig T^T: dL/dSig = T^T Gc T ; dL/dT = 2 Gc T Sig.
  double GSig[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int p = 0; p < 2; ++p)
        for (int r = 0; r < 2; ++r) a += T[3 * p + i] * Gc[2 * p + r] * T[3 * r + j];
      GSig[3 * i + j] = a;
    }
  double GT[6];
  for (int p = 0; p < 2; ++p)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) a += Gc[2 * p + r] * T[3 * r + k] * Sig[3 * k + j];
      GT[3 * p + j] = 2.0 * a;
    }
  // T = J Rc: dL/dJ = dL/dT Rc^T.
  double GJ[6];
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 3; ++k) {
      double a = 0;
      for (int j = 0; j < 3; ++j) a += GT[3 * p + j] * Rc[3 * k + j];
      GJ[3 * p + k] = a;
    }
  // J -> t (true derivative of the guard clamp).
  double gt[3] = {0, 0, 0};
  const double iz2 = iz * iz, iz3 = iz2 * iz;
  const double dtxc_dtx = clx ? 0.0 : 1.0, dtxc_dtz = clx ? cvx : 0.0;
  const double dtyc_dty = cly ? 0.0 : 1.0, dtyc_dtz = cly ? cvy : 0.0;
  gt[2] += GJ[0] * (-cam.fx * iz2) + GJ[4] * (-cam.fy * iz2);
  gt[0] += GJ[2] * (-cam.fx * iz2 * dtxc_dtx);
  gt[2] += GJ[2] * (-cam.fx * iz2 * dtxc_dtz + 2.0 * cam.fx * txc * iz3);
  gt[1] += GJ[5] * (-cam.fy * iz2 * dtyc_dty);
  gt[2] += GJ[5] * (-cam.fy * iz2 * dtyc_dtz + 2.0 * cam.fy * tyc * iz3);
  // Image-plane mean -> t.
  gt[0] += g2[0] * cam.fx * iz;
  gt[1] += g2[1] * cam.fy * iz;
  gt[2] += -g2[0] * cam.fx * t[0] * iz2 - g2[1] * cam.fy * t[1] * iz2;
  // t = Rc mean + tc.
  for (int j = 0; j < 3; ++j) gm[j] += Rc[j] * gt[0] + Rc[3 + j] * gt[1] + Rc[6 + j] * gt[2];

  // Sig = M M^T: dL/dM = 2 GSig M ; M = Rq diag(s).
  double GM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += GSig[3 * i + k] * M[3 * k + j];
      GM[3 * i + j] = 2.0 * a;
    }
  double GR[9];
  for (int j = 0; j < 3; ++j) {
    double gs = 0;
    for (int i = 0; i < 3; ++i) {
      gs += GM[3 * i + j] * Rq[3 * i + j];
      GR[3 * i + j] = GM[3 * i + j] * s[j];
    }
    gls[j] += gs * s[j];
  }
  double dR[4][9];
  quat_to_rot_grad(q, dR);
  double gqn[4];
  for (int c = 0; c < 4; ++c) {
    double a = 0;
    for (int e = 0; e < 9; ++e) a += GR[e] * dR[c][e];
    gqn[c] = a;
  }
  const double dotp = q[0] * gqn[0] + q[1] * gqn[1] + q[2] * gqn[2] + q[3] * gqn[3];
  for (int c = 0; c < 4; ++c) gq[c] += (gqn[c] - q[c] * dotp) / qn;

  // Opacity logit.
  const double op = po.rec[R_OP];
  *glogit += g2[5] * op * (1.0 - op);

  // Colour: SH coefficients and the viewing direction.
  const double cc[3] = {-(Rc[0] * cam.t[0] + Rc[3] * cam.t[1] + Rc[6] * cam.t[2]),
                        -(Rc[1] * cam.t[0] + Rc[4] * cam.t[1] + Rc[7] * cam.t[2]),
                        -(Rc[2] * cam.t[0] + Rc[5] * cam.t[1] + Rc[8] * cam.t[2])};
  double d[3] = {m[0] - cc[0], m[1] - cc[1], m[2] - cc[2]};
  const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  d[0] /= dn; d[1] /= dn; d[2] /= dn;
  double Y[16], GY[16][3];
  kSh.eval(D, d, Y, GY);
  double gd[3] = {0, 0, 0};
  for (int ch = 0; ch < 3; ++ch) {
    if (po.flags & (F_CLAMP_R << ch)) continue;
    const double gc = g2[6 + ch];
    for (int k = 0; k < sh_count(D); ++k) {
      gsh[3 * k + ch] += gc * Y[k];
      for (int e = 0; e < 3; ++e) gd[e] += gc * gi.sh[3 * k + ch] * GY[k][e];
    }
  }
  const double dd = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
  for (int e = 0; e < 3; ++e) gm[e] += (gd[e] - d[e] * dd) / dn;
}

GaussIn gauss_at(int64_t i, int D, const double* means, const double* ls, const double* quats, const double* logits,
                 const double* sh) {
  return {means + 3 * i, ls + 3 * i, quats + 4 * i, logits[i], sh + (size_t)i * sh_count(D) * 3};
}

}  // namespace

extern "C" {

int or_version(void) { return 1; }

// SH basis (and its polynomial gradient when grad != NULL) at n unit vectors.
void or_sh_basis(int32_t D, int64_t n, const double* dirs, double* Y, double* grad) {
  const int K = sh_count(D);
  for (int64_t i = 0; i < n; ++i) {
    double y[16], g[16][3];
    kSh.eval(D, dirs + 3 * i, y, grad ? g : nullptr);
    for (int k = 0; k < K; ++k) {
      Y[i * K + k] = y[k];
      if (grad)
        for (int e = 0; e < 3; ++e) grad[(i * K + k) * 3 + e] = g[k][e];
    }
  }
}

void or_quat_to_rot(const double* q_unit, double* R) { quat_to_rot(q_unit, R); }

// Projection of n Gaussians into one view.  Outputs per Gaussian: the record
// (mx, my, depth, conic a b c, opacity, r g b), radius r (0 = culled), the
// rect half-extents (rx, ry) (optional), tile rect (x0,y0,x1,y1), flag bits
// and the dilated 2D covariance (a, b, c) (optional).
int or_project(int64_t n, int32_t D, const double* means, const double* log_scales, const double* quats,
               const double* logits, const double* sh, const OrCamera* cam, const OrOptions* opt, double* rec,
               int32_t* radius, int32_t* ext, int32_t* rect, uint32_t* flags, double* cov) {
  if (D < 0 || D > 3 || n < 0) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    ProjOut po;
    project_one(gauss_at(i, D, means, log_scales, quats, logits, sh), D, *cam, *opt, po);
    std::memcpy(rec + i * R_STRIDE, po.rec, sizeof po.rec);
    radius[i] = po.radius;
    if (ext) std::memcpy(ext + 2 * i, po.ext, sizeof po.ext);
    std::memcpy(rect + 4 * i, po.rect, sizeof po.rect);
    flags[i] = po.flags;
    if (cov) std::memcpy(cov + 3 * i, po.cov, sizeof po.cov);
  }
  return 0;
}

// Tile binning and ordering: every (view, Gaussian) with half-extents
// (rx, ry), rx > 0, emits one pair per tile of its rect, in (view, Gaussian,
// tile) order, keyed by
// (global tile << 32) | FP32 bits of the depth; the pairs are stably sorted
// by key.  Inputs are FP32 records (either side's).  ranges[t] = [first,
// last+1) of tile t in the sorted arrays, (0,0) when empty.  Returns 2 and
// sets *n_pairs when the pair count exceeds capacity.
int or_bin(int32_t n_views, int64_t n, const float* mean2d, const int32_t* ext, const float* depth,
           const int32_t* wh, int32_t tile, int64_t capacity, uint64_t* keys, uint32_t* ids, uint32_t* ranges,
           int64_t* n_pairs) {
  std::vector<std::pair<uint64_t, uint32_t>> pairs;
  int64_t toff = 0;
  for (int v = 0; v < n_views; ++v) {
    const TileGrid g = grid_of(wh[2 * v], wh[2 * v + 1], tile);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t id = (int64_t)v * n + i;
      if (ext[2 * id] <= 0) continue;
      int r[4];
      tile_rect(mean2d[2 * id], mean2d[2 * id + 1], ext[2 * id], ext[2 * id + 1], tile, g, r);
      const uint32_t db = f32_bits(depth[id]);
      for (int ty = r[1]; ty < r[3]; ++ty)
        for (int tx = r[0]; tx < r[2]; ++tx) {
          const uint64_t gtile = (uint64_t)(toff + (int64_t)ty * g.tx + tx);
          pairs.push_back({(gtile << 32) | db, (uint32_t)id});
        }
    }
    toff += (int64_t)g.tx * g.ty;
  }
  *n_pairs = (int64_t)pairs.size();
  if ((int64_t)pairs.size() > capacity) return 2;
  std::stable_sort(pairs.begin(), pairs.end(),
                   [](const std::pair<uint64_t, uint32_t>& a, const std::pair<uint64_t, uint32_t>& b) {
                     return a.first < b.first;
                   });
  std::memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)toff);
  for (size_t p = 0; p < pairs.size(); ++p) {
    if (keys) keys[p] = pairs[p].first;
    ids[p] = pairs[p].second;
    const uint64_t t = pairs[p].first >> 32;
    if (p == 0 || (pairs[p - 1].first >> 32) != t) ranges[2 * t] = (uint32_t)p;
    ranges[2 * t + 1] = (uint32_t)(p + 1);
  }
  return 0;
}

int or_render_tiles(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
                    const uint32_t* ids, const uint32_t* ranges, const int64_t* tiles, int64_t n_tiles, double* image,
                    double* t_final, int32_t* n_contrib, uint32_t* pix_flags);

// Forward render of all views from records [V*N][10] and sorted tile lists.
// image is [sum_v 3*H_v*W_v] (view-major, planar channels), t_final and
// n_contrib [sum_v H_v*W_v]; pix_flags marks near-threshold decisions.
int or_render(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
              const uint32_t* ids, const uint32_t* ranges, double* image, double* t_final, int32_t* n_contrib,
              uint32_t* pix_flags) {
  return or_render_tiles(n_views, n, cams, opt, rec, ids, ranges, nullptr, -1, image, t_final, n_contrib, pix_flags);
}

// As or_render, restricted to the listed global tiles (all tiles when `tiles`
// is NULL); pixels of other tiles are left untouched.
int or_render_tiles(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
                    const uint32_t* ids, const uint32_t* ranges, const int64_t* tiles, int64_t n_tiles, double* image,
                    double* t_final, int32_t* n_contrib, uint32_t* pix_flags) {
  (void)n;
  const std::vector<ViewInfo> views = make_views(cams, n_views, opt->tile);
  const int64_t T_tot = views.back().tile_off + (int64_t)views.back().grid.tx * views.back().grid.ty;
  const int B = opt->tile;
  const int64_t count = tiles ? n_tiles : T_tot;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t ti = 0; ti < count; ++ti) {
    const int64_t gt = tiles ? tiles[ti] : ti;
    const int v = view_of_tile(views, gt);
    const ViewInfo& vw = views[v];
    const int64_t lt = gt - vw.tile_off;
    const int tx = (int)(lt % vw.grid.tx), ty = (int)(lt / vw.grid.tx);
    const uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];
    const int W = vw.cam.width, H = vw.cam.height;
    PixelTrace tr;
    for (int j = ty * B; j < std::min(H, (ty + 1) * B); ++j)
      for (int i = tx * B; i < std::min(W, (tx + 1) * B); ++i) {
        trace_pixel(i, j, ids + s, (int64_t)e - s, rec, *opt, false, tr);
        const int64_t p = vw.pix_off + (int64_t)j * W + i;
        for (int ch = 0; ch < 3; ++ch)
          image[3 * vw.pix_off + (int64_t)ch * W * H + (int64_t)j * W + i] = tr.C[ch] + tr.T * opt->bg[ch];
        if (t_final) t_final[p] = tr.T;
        if (n_contrib) n_contrib[p] = tr.n_contrib;
        if (pix_flags) pix_flags[p] = tr.flags;
      }
  }
  return 0;
}

// Backward of the blending restricted to the listed global tiles (all when
// `tiles` is NULL): grad2d [V*N][9] receives the image-space gradients summed
// over the pixels of those tiles only, and abs2d [V*N][2] (when not NULL) the
// per-pixel magnitudes of the two mean components summed the same way.
// A decision of one pixel taken the other way (see Flip): pixel = global pixel index.
struct PixelFlip {
  int64_t pixel;
  Flip flip;
};

static int render_backward_impl(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt,
                                const double* rec, const uint32_t* ids, const uint32_t* ranges, const int64_t* tiles,
                                int64_t n_tiles, const double* dl_dimage, double* grad2d, double* abs2d,
                                const std::vector<PixelFlip>* flips = nullptr, double* mag9 = nullptr) {
  const std::vector<ViewInfo> views = make_views(cams, n_views, opt->tile);
  const int64_t T_tot = views.back().tile_off + (int64_t)views.back().grid.tx * views.back().grid.ty;
  const int B = opt->tile;
  const int64_t count = tiles ? n_tiles : T_tot;
  // per selected tile, one gradient row per list entry (summed over the tile's pixels)
  std::vector<int64_t> row_off(count + 1, 0);
  for (int64_t ti = 0; ti < count; ++ti) {
    const int64_t gt = tiles ? tiles[ti] : ti;
    row_off[ti + 1] = row_off[ti] + (int64_t)ranges[2 * gt + 1] - (int64_t)ranges[2 * gt];
  }
  std::vector<double> rows((size_t)row_off[count] * kRowW, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t ti = 0; ti < count; ++ti) {
    const int64_t gt = tiles ? tiles[ti] : ti;
    const int v = view_of_tile(views, gt);
    const ViewInfo& vw = views[v];
    const int64_t lt = gt - vw.tile_off;
    const int tx = (int)(lt % vw.grid.tx), ty = (int)(lt / vw.grid.tx);
    const uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];
    const int W = vw.cam.width, H = vw.cam.height;
    PixelTrace tr;
    for (int j = ty * B; j < std::min(H, (ty + 1) * B); ++j)
      for (int i = tx * B; i < std::min(W, (tx + 1) * B); ++i) {
        Flip f;
        if (flips && !flips->empty()) {
          const int64_t p = vw.pix_off + (int64_t)j * W + i;
          auto it = std::lower_bound(flips->begin(), flips->end(), p,
                                     [](const PixelFlip& a, int64_t q) { return a.pixel < q; });
          if (it != flips->end() && it->pixel == p) f = it->flip;
        }
        trace_pixel(i, j, ids + s, (int64_t)e - s, rec, *opt, true, tr, 0xffffffffu, nullptr, f);
        double dl[3];
        for (int ch = 0; ch < 3; ++ch) dl[ch] = dl_dimage[3 * vw.pix_off + (int64_t)ch * W * H + (int64_t)j * W + i];
        backward_pixel(tr, dl, rec, *opt, rows.data() + (size_t)row_off[ti] * kRowW);
      }
  }
  std::memset(grad2d, 0, sizeof(double) * 9 * (size_t)n_views * n);
  if (abs2d) std::memset(abs2d, 0, sizeof(double) * 2 * (size_t)n_views * n);
  if (mag9) std::memset(mag9, 0, sizeof(double) * 9 * (size_t)n_views * n);
  for (int64_t ti = 0; ti < count; ++ti) {
    const int64_t gt = tiles ? tiles[ti] : ti;
    const uint32_t s = ranges[2 * gt];
    for (int64_t k = 0; k < row_off[ti + 1] - row_off[ti]; ++k) {
      const double* row = rows.data() + (size_t)(row_off[ti] + k) * kRowW;
      for (int c = 0; c < 9; ++c) grad2d[(size_t)ids[s + k] * 9 + c] += row[c];
      if (abs2d)
        for (int c = 0; c < 2; ++c) abs2d[(size_t)ids[s + k] * 2 + c] += row[9 + c];
      if (mag9)
        for (int c = 0; c < 9; ++c) mag9[(size_t)ids[s + k] * 9 + c] += row[11 + c];
    }
  }
  return 0;
}

int or_render_backward_tiles(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt,
                             const double* rec, const uint32_t* ids, const uint32_t* ranges, const int64_t* tiles,
                             int64_t n_tiles, const double* dl_dimage, double* grad2d) {
  return render_backward_impl(n_views, n, cams, opt, rec, ids, ranges, tiles, n_tiles, dl_dimage, grad2d, nullptr);
}

// As or_render_backward_tiles, with one decision of each listed pixel taken
// the other way: pixel flip_px[q] (global index, ascending, distinct) takes
// the decision of kind flip_kind[q] (a P_NEAR_* bit) at list position
// flip_k[q] the other way.  For comparing with an FP32 evaluation that went
// the other way at near-threshold decisions.  mag9 [V*N][9] (may be NULL)
// receives, per row and component, the sum over pixels of the magnitudes of
// the parts of the per-pixel terms that grad2d adds up (see backward_pixel).
int or_render_backward_tiles_flips(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt,
                                   const double* rec, const uint32_t* ids, const uint32_t* ranges,
                                   const int64_t* tiles, int64_t n_tiles, const double* dl_dimage, double* grad2d,
                                   int64_t n_flips, const int64_t* flip_px, const int32_t* flip_k,
                                   const uint32_t* flip_kind, double* mag9) {
  std::vector<PixelFlip> flips((size_t)n_flips);
  for (int64_t q = 0; q < n_flips; ++q) {
    if (q > 0 && flip_px[q] <= flip_px[q - 1]) return 1;
    flips[q].pixel = flip_px[q];
    flips[q].flip.k = flip_k[q];
    flips[q].flip.kind = flip_kind[q];
  }
  return render_backward_impl(n_views, n, cams, opt, rec, ids, ranges, tiles, n_tiles, dl_dimage, grad2d, nullptr,
                              &flips, mag9);
}

// The backward of the blending over all tiles with the homodirectional
// view-space gradient of AbsGS (Sec. III-B adaptive control): abs2d [V*N][2]
// = per (view, Gaussian) the sum over pixels of |dL_pixel/dmx| and
// |dL_pixel/dmy| (pixel units), where dL_pixel is the loss through that
// pixel's colour alone.
int or_render_backward_abs(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
                           const uint32_t* ids, const uint32_t* ranges, const double* dl_dimage, double* grad2d,
                           double* abs2d) {
  return render_backward_impl(n_views, n, cams, opt, rec, ids, ranges, nullptr, -1, dl_dimage, grad2d, abs2d);
}

// Backward of the blending: given dL/dimage (same layout as the image), the
// 9 image-space gradients per (view, Gaussian) in grad2d [V*N][9], order
// (mx, my, conic a, b, c, opacity, r, g, b).  Summation over pixels is in a
// fixed order (tile by tile, pixel by pixel).
int or_render_backward(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
                       const uint32_t* ids, const uint32_t* ranges, int64_t n_pairs, const double* dl_dimage,
                       double* grad2d) {
  (void)n_pairs;
  return or_render_backward_tiles(n_views, n, cams, opt, rec, ids, ranges, nullptr, -1, dl_dimage, grad2d);
}

// Chain image-space gradients [V*N][9] to the raw parameters, summed over
// views in view order.  Outputs are overwritten.
int or_project_backward(int64_t n, int32_t D, const double* means, const double* log_scales, const double* quats,
                        const double* logits, const double* sh, const OrCamera* cams, int32_t n_views,
                        const OrOptions* opt, const double* grad2d, double* g_means, double* g_log_scales,
                        double* g_quats, double* g_logits, double* g_sh) {
  const int K = sh_count(D);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double gm[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gl = 0;
    std::vector<double> gsh((size_t)K * 3, 0.0);
    const GaussIn gi = gauss_at(i, D, means, log_scales, quats, logits, sh);
    for (int v = 0; v < n_views; ++v)
      project_backward_one(gi, D, cams[v], *opt, grad2d + ((size_t)v * n + i) * 9, gm, gls, gq, &gl, gsh.data());
    std::memcpy(g_means + 3 * i, gm, sizeof gm);
    std::memcpy(g_log_scales + 3 * i, gls, sizeof gls);
    std::memcpy(g_quats + 4 * i, gq, sizeof gq);
    g_logits[i] = gl;
    std::memcpy(g_sh + (size_t)i * K * 3, gsh.data(), sizeof(double) * K * 3);
  }
  return 0;
}

// Central finite differences of the L1 loss
//   L = sum_v 1/(3 H_v W_v) sum_{pixels, channels} |C - target|
// with respect to single raw parameters, re-rendering only the tiles whose
// lists can change (those covered by the perturbed Gaussian before or after
// the step).  Parameter index p of Gaussian g: 0-2 mean, 3-5 log-scale,
// 6-9 quaternion, 10 opacity logit, 11.. SH coefficient (k*3 + channel).
// status[s]: 0 = accepted at h, 1 = accepted at h/10, 2 = the discrete
// structure (blended set, order, stop point, clamps, L1 signs) changed.
int or_fd_local(int64_t n, int32_t D, const double* means, const double* log_scales, const double* quats,
                const double* logits, const double* sh, const OrCamera* cams, int32_t n_views, const OrOptions* opt,
                const double* target, int64_t n_samples, const int64_t* sample_g, const int32_t* sample_p,
                double h_rel, double* fd, int32_t* status) {
  const int K = sh_count(D);
  const int B = opt->tile;
  const std::vector<ViewInfo> views = make_views(cams, n_views, B);
  // Base projection and per-tile lists (pair key = depth bits, id).
  std::vector<double> rec((size_t)n_views * n * R_STRIDE);
  std::vector<int32_t> rad((size_t)n_views * n), rect((size_t)n_views * n * 4);
  for (int v = 0; v < n_views; ++v) {
    std::vector<uint32_t> fl(n);
    or_project(n, D, means, log_scales, quats, logits, sh, &cams[v], opt, rec.data() + (size_t)v * n * R_STRIDE,
               rad.data() + (size_t)v * n, nullptr, rect.data() + (size_t)v * n * 4, fl.data(), nullptr);
  }
  const int64_t T_tot = views.back().tile_off + (int64_t)views.back().grid.tx * views.back().grid.ty;
  std::vector<std::vector<std::pair<uint32_t, uint32_t>>> lists(T_tot);
  for (int v = 0; v < n_views; ++v)
    for (int64_t i = 0; i < n; ++i) {
      const size_t id = (size_t)v * n + i;
      if (rad[id] <= 0) continue;
      const int* r = &rect[id * 4];
      const uint32_t db = f32_bits((float)rec[id * R_STRIDE + R_DEPTH]);
      for (int ty = r[1]; ty < r[3]; ++ty)
        for (int tx = r[0]; tx < r[2]; ++tx)
          lists[views[v].tile_off + (int64_t)ty * views[v].grid.tx + tx].push_back({db, (uint32_t)id});
    }
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t t = 0; t < T_tot; ++t) std::stable_sort(lists[t].begin(), lists[t].end(),
                                                        [](const std::pair<uint32_t, uint32_t>& a,
                                                           const std::pair<uint32_t, uint32_t>& b) { return a.first < b.first; });

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t si = 0; si < n_samples; ++si) {
    const int64_t g = sample_g[si];
    const int p = sample_p[si];
    double pm[3], pls[3], pq[4], pl;
    std::vector<double> psh((size_t)K * 3);
    auto load = [&]() {
      std::memcpy(pm, means + 3 * g, sizeof pm);
      std::memcpy(pls, log_scales + 3 * g, sizeof pls);
      std::memcpy(pq, quats + 4 * g, sizeof pq);
      pl = logits[g];
      std::memcpy(psh.data(), sh + (size_t)g * K * 3, sizeof(double) * K * 3);
    };
    auto param = [&](int idx) -> double& {
      if (idx < 3) return pm[idx];
      if (idx < 6) return pls[idx - 3];
      if (idx < 10) return pq[idx - 6];
      if (idx == 10) return pl;
      return psh[idx - 11];
    };
    load();
    const double theta = param(p);
    // Evaluate the weighted per-pixel residuals of the affected tiles and a
    // signature of the discrete structure.  The two one-sided evaluations are
    // differenced residual by residual, which keeps the rounding error of the
    // quotient far below that of differencing two loss totals.
    auto eval = [&](double h, const std::vector<int64_t>& tiles, std::vector<double>& res, uint64_t& sig) {
      load();
      param(p) = theta + h;
      GaussIn gi{pm, pls, pq, pl, psh.data()};
      std::vector<ProjOut> pv(n_views);
      res.clear();
      sig = 1469598103934665603ull;
      auto mix = [&](uint64_t x) { sig = (sig ^ x) * 1099511628211ull; };
      for (int v = 0; v < n_views; ++v) {
        project_one(gi, D, views[v].cam, *opt, pv[v]);
        mix((uint64_t)pv[v].flags & 0xfffu);
      }
      PixelTrace tr;
      for (size_t ti = 0; ti < tiles.size(); ++ti) {
        const int64_t gtile = tiles[ti];
        const int v = view_of_tile(views, gtile);
        const ViewInfo& vw = views[v];
        const ProjOut& po = pv[v];
        const uint32_t gid = (uint32_t)((size_t)v * n + g);
        const int64_t lt = gtile - vw.tile_off;
        const int tx = (int)(lt % vw.grid.tx), ty = (int)(lt / vw.grid.tx);
        const bool covers = po.radius > 0 && tx >= po.rect[0] && tx < po.rect[2] && ty >= po.rect[1] && ty < po.rect[3];
        // Local list: base list without g, plus g at its key position.
        std::vector<std::pair<uint32_t, uint32_t>> L;
        L.reserve(lists[gtile].size() + 1);
        for (auto& e : lists[gtile])
          if (e.second != gid) L.push_back(e);
        if (covers) {
          std::pair<uint32_t, uint32_t> me{f32_bits((float)po.rec[R_DEPTH]), gid};
          auto it = std::upper_bound(L.begin(), L.end(), me,
                                     [](const std::pair<uint32_t, uint32_t>& a, const std::pair<uint32_t, uint32_t>& b) {
                                       return a.first < b.first || (a.first == b.first && a.second < b.second);
                                     });
          L.insert(it, me);
        }
        std::vector<uint32_t> ids(L.size());
        for (size_t k = 0; k < L.size(); ++k) { ids[k] = L[k].second; mix(L[k].second); }
        const int W = vw.cam.width, H = vw.cam.height;
        const double wgt = 1.0 / (3.0 * W * H);
        for (int j = ty * B; j < std::min(H, (ty + 1) * B); ++j)
          for (int i = tx * B; i < std::min(W, (tx + 1) * B); ++i) {
            trace_pixel(i, j, ids.data(), (int64_t)ids.size(), rec.data(), *opt, true, tr, gid, po.rec);
            for (auto& a : tr.acc) mix(((uint64_t)a.k << 1) | (a.clamped ? 1u : 0u));
            mix((uint64_t)(tr.stop_k + 1));
            for (int ch = 0; ch < 3; ++ch) {
              const double c = tr.C[ch] + tr.T * opt->bg[ch];
              const double d = c - target[3 * vw.pix_off + (int64_t)ch * W * H + (int64_t)j * W + i];
              res.push_back(wgt);
              res.push_back(d);
              mix(d > 0 ? 1u : (d < 0 ? 2u : 3u));
            }
          }
      }
    };
    int st = 2;
    double hv = h_rel * std::max(1.0, std::fabs(theta));
    for (int attempt = 0; attempt < 2 && st == 2; ++attempt, hv *= 0.1) {
      // Affected tiles: union of g's rects at theta, theta+h, theta-h in every view.
      std::vector<int64_t> tiles;
      for (int sgn = -1; sgn <= 1; ++sgn) {
        load();
        param(p) = theta + sgn * hv;
        GaussIn gi{pm, pls, pq, pl, psh.data()};
        for (int v = 0; v < n_views; ++v) {
          ProjOut po;
          project_one(gi, D, views[v].cam, *opt, po);
          if (po.radius <= 0) continue;
          for (int ty = po.rect[1]; ty < po.rect[3]; ++ty)
            for (int tx = po.rect[0]; tx < po.rect[2]; ++tx)
              tiles.push_back(views[v].tile_off + (int64_t)ty * views[v].grid.tx + tx);
        }
      }
      std::sort(tiles.begin(), tiles.end());
      tiles.erase(std::unique(tiles.begin(), tiles.end()), tiles.end());
      std::vector<double> rp, rm;
      uint64_t sp, sm;
      eval(+hv, tiles, rp, sp);
      eval(-hv, tiles, rm, sm);
      double diff = 0;
      for (size_t k = 0; k + 1 < rp.size() && k + 1 < rm.size(); k += 2)
        diff += rp[k] * (std::fabs(rp[k + 1]) - std::fabs(rm[k + 1]));
      fd[si] = diff / (2.0 * hv);
      st = (sp == sm) ? attempt : 2;
    }
    status[si] = st;
  }
  return 0;
}

// Per-pixel work of the blending: list entries evaluated until the pixel
// stops (list end, or the entry that would take T below t_min, inclusive)
// and entries blended.  Same inputs as or_render; outputs [sum_v H_v*W_v].
int or_pixel_counts(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
                    const uint32_t* ids, const uint32_t* ranges, int64_t* evaluated, int64_t* blended) {
  (void)n;
  const std::vector<ViewInfo> views = make_views(cams, n_views, opt->tile);
  const int64_t T_tot = views.back().tile_off + (int64_t)views.back().grid.tx * views.back().grid.ty;
  const int B = opt->tile;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t gt = 0; gt < T_tot; ++gt) {
    const int v = view_of_tile(views, gt);
    const ViewInfo& vw = views[v];
    const int64_t lt = gt - vw.tile_off;
    const int tx = (int)(lt % vw.grid.tx), ty = (int)(lt / vw.grid.tx);
    const uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];
    const int W = vw.cam.width, H = vw.cam.height;
    PixelTrace tr;
    for (int j = ty * B; j < std::min(H, (ty + 1) * B); ++j)
      for (int i = tx * B; i < std::min(W, (tx + 1) * B); ++i) {
        trace_pixel(i, j, ids + s, (int64_t)e - s, rec, *opt, true, tr);
        const int64_t p = vw.pix_off + (int64_t)j * W + i;
        evaluated[p] = tr.stop_k >= 0 ? tr.stop_k + 1 : (int64_t)e - s;
        blended[p] = (int64_t)tr.acc.size();
      }
  }
  return 0;
}


// Tile binning of a sample of tiles, by the same brute force as or_bin: every
// pair with rx > 0 is tested against the tiles of its rect, in (view,
// Gaussian) order.  tile_count [T_tot] receives the number of incidences of
// every tile; for the listed tiles (ascending, distinct) the ids covering
// each, stably sorted by the FP32 bits of their depth (so ties stay in id
// order), are concatenated in list order into out_ids (capacity out_cap) and
// out_len [n_tiles] receives each list's length.  Returns 2 when out_cap is
// too small.  For workloads whose full binning does not fit in memory.
int or_bin_sampled(int32_t n_views, int64_t n, const float* mean2d, const int32_t* ext, const float* depth,
                   const int32_t* wh, int32_t tile, const int64_t* tiles, int64_t n_tiles, int64_t* tile_count,
                   uint32_t* out_ids, int64_t out_cap, int64_t* out_len) {
  int64_t T_tot = 0;
  for (int v = 0; v < n_views; ++v) {
    const TileGrid g = grid_of(wh[2 * v], wh[2 * v + 1], tile);
    T_tot += (int64_t)g.tx * g.ty;
  }
  std::vector<int64_t> slot(T_tot, -1);  // sample index of a global tile
  for (int64_t k = 0; k < n_tiles; ++k) slot[tiles[k]] = k;
  std::vector<std::vector<std::pair<uint32_t, uint32_t>>> lists(n_tiles);  // (depth bits, id)
  std::memset(tile_count, 0, sizeof(int64_t) * (size_t)T_tot);
  int64_t toff = 0;
  for (int v = 0; v < n_views; ++v) {
    const TileGrid g = grid_of(wh[2 * v], wh[2 * v + 1], tile);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t id = (int64_t)v * n + i;
      if (ext[2 * id] <= 0) continue;
      int r[4];
      tile_rect(mean2d[2 * id], mean2d[2 * id + 1], ext[2 * id], ext[2 * id + 1], tile, g, r);
      for (int ty = r[1]; ty < r[3]; ++ty)
        for (int tx = r[0]; tx < r[2]; ++tx) {
          const int64_t gt = toff + (int64_t)ty * g.tx + tx;
          ++tile_count[gt];
          if (slot[gt] >= 0) lists[slot[gt]].push_back({f32_bits(depth[id]), (uint32_t)id});
        }
    }
    toff += (int64_t)g.tx * g.ty;
  }
  int64_t o = 0;
  for (int64_t k = 0; k < n_tiles; ++k) {
    auto& l = lists[k];
    std::stable_sort(l.begin(), l.end(), [](const std::pair<uint32_t, uint32_t>& a,
                                            const std::pair<uint32_t, uint32_t>& b) { return a.first < b.first; });
    out_len[k] = (int64_t)l.size();
    if (o + (int64_t)l.size() > out_cap) return 2;
    for (const auto& e : l) out_ids[o++] = e.second;
  }
  return 0;
}

// Locate pixel p (global index over the packed views) in the views.
static void locate_pixel(const std::vector<ViewInfo>& views, int B, int64_t p, int* v_out, int* i_out, int* j_out,
                         int64_t* gt_out) {
  int v = 0;
  while (v + 1 < (int)views.size() && views[v + 1].pix_off <= p) ++v;
  const ViewInfo& vw = views[v];
  const int64_t lp = p - vw.pix_off;
  const int W = vw.cam.width;
  const int i = (int)(lp % W), j = (int)(lp / W);
  *v_out = v;
  *i_out = i;
  *j_out = j;
  *gt_out = vw.tile_off + (int64_t)(j / B) * vw.grid.tx + i / B;
}

// One-flip alternatives of listed pixels: for pixel pixels[q] (global index),
// n_alt[q] receives the number of its near-threshold decisions (or -1 when
// there are more than max_alt, or more than the trace keeps), and alt
// [n_pix][max_alt][3] the colour (background included) the pixel takes when
// exactly the a-th of them goes the other way, every other decision as
// defined; kinds [n_pix][max_alt] the P_NEAR_* bit of each and ks its list
// position.  A value computed
// with FP32 arithmetic near such a threshold may take either side of it.
int or_render_flips(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
                    const uint32_t* ids, const uint32_t* ranges, const int64_t* pixels, int64_t n_pix, int32_t max_alt,
                    int32_t* n_alt, double* alt, uint32_t* kinds, int32_t* ks) {
  (void)n;
  const std::vector<ViewInfo> views = make_views(cams, n_views, opt->tile);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_pix; ++q) {
    int v, i, j;
    int64_t gt;
    locate_pixel(views, opt->tile, pixels[q], &v, &i, &j, &gt);
    const uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];
    PixelTrace tr, tf;
    trace_pixel(i, j, ids + s, (int64_t)e - s, rec, *opt, false, tr);
    const int nf = tr.n_flagged;
    n_alt[q] = (nf > max_alt || nf > kMaxFlagged) ? -1 : nf;
    for (int a = 0; a < std::min(nf, std::min<int>(max_alt, kMaxFlagged)); ++a) {
      Flip f;
      f.k = tr.flagged[a].k;
      f.kind = tr.flagged[a].kind;
      trace_pixel(i, j, ids + s, (int64_t)e - s, rec, *opt, false, tf, 0xffffffffu, nullptr, f);
      for (int ch = 0; ch < 3; ++ch) alt[(q * max_alt + a) * 3 + ch] = tf.C[ch] + tf.T * opt->bg[ch];
      kinds[q * max_alt + a] = f.kind;
      ks[q * max_alt + a] = f.k;
    }
  }
  return 0;
}

// Discrete decisions of every pixel, for comparing two renders of the same
// scene whose records or lists come from different projections: per pixel
// the number of blended entries, an order-independent hash of their ids
// (sum of a 64-bit mix of each id), the id that ended the pixel (0xffffffff
// when none), and the smallest relative distance of any evaluated entry's
// alpha from alpha_min and of any blended or stopping entry's transmittance
// from t_min (how far the closest threshold decision was).
int or_pixel_decisions(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
                       const uint32_t* ids, const uint32_t* ranges, int32_t* n_blended, uint64_t* blend_hash,
                       uint32_t* stop_id, double* margin_alpha, double* margin_t) {
  (void)n;
  const std::vector<ViewInfo> views = make_views(cams, n_views, opt->tile);
  const int64_t T_tot = views.back().tile_off + (int64_t)views.back().grid.tx * views.back().grid.ty;
  const int B = opt->tile;
  auto mix = [](uint64_t x) {  // splitmix64 finaliser
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
  };
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t gt = 0; gt < T_tot; ++gt) {
    const int v = view_of_tile(views, gt);
    const ViewInfo& vw = views[v];
    const int64_t lt = gt - vw.tile_off;
    const int tx = (int)(lt % vw.grid.tx), ty = (int)(lt / vw.grid.tx);
    const uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];
    const int W = vw.cam.width, H = vw.cam.height;
    PixelTrace tr;
    for (int j = ty * B; j < std::min(H, (ty + 1) * B); ++j)
      for (int i = tx * B; i < std::min(W, (tx + 1) * B); ++i) {
        trace_pixel(i, j, ids + s, (int64_t)e - s, rec, *opt, true, tr);
        const int64_t p = vw.pix_off + (int64_t)j * W + i;
        uint64_t h = 0;
        for (const Accepted& a : tr.acc) h += mix(a.id);
        n_blended[p] = (int32_t)tr.acc.size();
        blend_hash[p] = h;
        stop_id[p] = tr.stop_k >= 0 ? ids[s + tr.stop_k] : 0xffffffffu;
        margin_alpha[p] = tr.margin_alpha;
        margin_t[p] = tr.margin_t;
      }
  }
  return 0;
}


// The single decision, taken the other way, that gives listed pixel q the
// contributor count target_nc[q] and the final transmittance target_T[q]
// (within 1e-3 relative; an FP32 evaluation that went the other way at some
// threshold shows in both: a blended entry scales T by 1 - alpha, at least
// 1/255 away from 1): candidates are the four threshold tests at every list
// position up to two past the larger of the defined and target counts and of
// the stop position; among those reaching both targets, the one whose colour
// is nearest target_rgb[q] (3 per pixel).  found[q] = 0 when the defined
// decisions already give both targets, 1 with (flip_k[q], flip_kind[q]) set,
// -1 when no single flip does.
int or_find_flips(int32_t n_views, int64_t n, const OrCamera* cams, const OrOptions* opt, const double* rec,
                  const uint32_t* ids, const uint32_t* ranges, const int64_t* pixels, int64_t n_pix,
                  const int32_t* target_nc, const double* target_T, const double* target_rgb, int32_t* found,
                  int32_t* flip_k, uint32_t* flip_kind) {
  (void)n;
  const std::vector<ViewInfo> views = make_views(cams, n_views, opt->tile);
  const uint32_t kinds[4] = {P_NEAR_ALPHA_MIN, P_NEAR_T_MIN, P_NEAR_POWER0, P_NEAR_ALPHA_MAX};
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < n_pix; ++q) {
    int v, i, j;
    int64_t gt;
    locate_pixel(views, opt->tile, pixels[q], &v, &i, &j, &gt);
    const uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];
    const int64_t len = (int64_t)e - s;
    PixelTrace tr, tf;
    trace_pixel(i, j, ids + s, len, rec, *opt, false, tr);
    found[q] = 0;
    flip_k[q] = -1;
    flip_kind[q] = 0;
    auto same_T = [&](double T) { return std::fabs(T - target_T[q]) <= 1e-3 * target_T[q]; };
    if (tr.n_contrib == target_nc[q] && same_T(tr.T)) continue;
    const int64_t hi = std::min<int64_t>(len - 1, (int64_t)std::max({tr.n_contrib, target_nc[q], tr.stop_k}) + 2);
    double best = INFINITY;
    found[q] = -1;
    for (int64_t k = 0; k <= hi; ++k)
      for (uint32_t kind : kinds) {
        Flip f;
        f.k = (int)k;
        f.kind = kind;
        trace_pixel(i, j, ids + s, len, rec, *opt, false, tf, 0xffffffffu, nullptr, f);
        if (tf.n_contrib != target_nc[q] || !same_T(tf.T)) continue;
        double d = std::fabs(tf.T - target_T[q]) / target_T[q];
        for (int ch = 0; ch < 3; ++ch)
          d = std::max(d, std::fabs(tf.C[ch] + tf.T * opt->bg[ch] - target_rgb[3 * q + ch]));
        if (d < best) {
          best = d;
          found[q] = 1;
          flip_k[q] = (int)k;
          flip_kind[q] = kind;
        }
      }
  }
  return 0;
}

// Thread count of the OpenMP loops (the CPU-baseline leg times the oracle at
// one thread and at all cores); returns the count in force afterwards.
int32_t or_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

}  // extern "C"
