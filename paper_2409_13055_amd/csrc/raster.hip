// Tile rasteriser: front-to-back blending (Sec. II) of the depth-ordered
// splat list of each screen tile, its backward pass, and the L1 term of the
// photometric loss, eq. (2).
//
// Work decomposition (gfx950, wave64): one workgroup per screen tile.  A
// 16x16 tile is ONE wavefront whose lanes own a column of 4 vertically
// adjacent pixels each; an 8x8 tile is one wavefront with one pixel per lane;
// a 32x32 tile is four wavefronts of 4 pixels per lane.  Splat records are
// staged in LDS in batches of one record per lane and read back as
// broadcasts (every lane reads the same address: no bank conflicts).  In the
// backward pass each lane first sums its own pixels, then the wavefront
// reduces the 9 image-space gradient terms with DPP row operations and the
// gfx950 permlane16/32 swaps, and 9 lanes issue one hardware FP32 atomic each,
// so one atomic per term per wavefront per splat reaches L2.
#include <algorithm>
#include <mutex>
#include <string>

#include "gs_internal.h"

namespace gs {

gs_status validate_params(const gs_params* p);
gs_status launch_project_bwd(const gs_params* params, const gs_camera* cams, int32_t n_views, const gs_options* opts,
                             const int32_t* tiles, const float* grad2d, const gs_grads* grads, hipStream_t stream);

struct RasterConsts {
  float alpha_min, alpha_max, t_min;
  float bg0, bg1, bg2;
  float radius_sigmas;
};

// The per-pixel exponent power = -(a dx^2 + c dy^2)/2 - b dx dy, d = pixel -
// mean, is evaluated in base 2 and with the opposite sign: the conic is scaled
// by log2(e) when an entry is staged (kLog2e below), and the kernels form
// q = -log2(e) power >= 0, so alpha = o exp2(-q) with no multiply per pixel.
// One fixed rounding sequence, ((c'/2) dy + b' dx) dy + (a'/2) dx^2 with the
// scaled coefficients (the dx terms shared by the PPL pixels of a lane's
// column), makes every kernel take identical decisions.  Rounding is symmetric,
// so q is exactly -log2(e) power as the opposite signs would give it, except
// that an exact zero comes out as +0.  With q >= 0 the test "power in
// [cutoff, 0]" is one unsigned comparison of bit patterns: bits(q) <=
// bits(qmax) for a staged qmax >= 0 holds exactly for +0 <= q <= qmax, and
// fails for a negative q (power > 0), +inf and NaN.
struct RowTerms {
  float a2x, bx;  // a dx^2 / 2 and b dx (scaled)
};
__device__ __forceinline__ RowTerms row_terms(float dx, float a2, float b) {
#pragma clang fp contract(off)
  return RowTerms{(a2 * dx) * dx, b * dx};
}
__device__ __forceinline__ float splat_q(const RowTerms& t, float c2, float dy) {
#pragma clang fp contract(off)
  return fmaf(fmaf(c2, dy, t.bx), dy, t.a2x);
}
__device__ __forceinline__ bool q_in_range(float q, float qmax) {
  return __float_as_uint(q) <= __float_as_uint(qmax);
}

// Below this (natural) exponent opacity * exp(power) < alpha_min is certain:
// the 1e-3 margin in the exponent covers the rounding of the logarithm, of the
// base-2 scaling, of exp2 and of the product, so skipping such entries before
// exp2 changes no decision.  The staged bound is qmax = max(0, -log2(e)
// cutoff): an entry whose opacity is below alpha_min, or NaN, keeps only q = +0,
// where alpha = opacity fails the alpha_min test (and the wave-level cull has
// already dropped it).
__device__ __forceinline__ float power_cutoff(float opacity, float alpha_min) {
  return __logf(alpha_min / opacity) - 1.0e-3f;
}

constexpr float kLog2e = 1.4426950408889634f;  // the staged conic and cutoff are in base 2
constexpr float kLn2 = 0.6931471805599453f;    // back to natural units (the conic's gradient factors)

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}

// Sum over the 64 lanes of a wavefront; every lane receives the total.
__device__ __forceinline__ float wave_sum(float x) {
  x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp<0x141>(x);  // row_half_mirror
  x += dpp<0x140>(x);  // row_mirror: each 16-lane row now holds its row sum
  const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  x = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
  const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r32[0]) + __uint_as_float(r32[1]);
}

// Wavefront layout of a tile's workgroup: WAVES wavefronts of PPL pixels per lane.
template <int W, int P>
struct Shape {
  static constexpr int WAVES = W, PPL = P, THREADS = 64 * W;
};
// Forward and work counts: one 8x8 wave at tile 8, one 16x16 wave of 4 px/lane at tile 16,
// four 16x16 waves at tile 32.
template <int TILE>
struct FwdShape;
template <>
struct FwdShape<8> : Shape<1, 1> {};
template <>
struct FwdShape<16> : Shape<1, 4> {};
template <>
struct FwdShape<32> : Shape<4, 4> {};
// Backward: at tile 32, two 16x32 waves of 8 px/lane.  A splat that covers the tile is then
// walked, tested and reduced by two waves instead of four, which halves the per-entry work
// (about a third of the backward's instructions); the lighter forward loses more to the lower
// occupancy that eight pixels per lane bring than it gains.  The per-pixel arithmetic does not
// depend on the layout, so both kernels still decide identically for every pixel.
template <int TILE>
struct BwdShape : FwdShape<TILE> {};
template <>
struct BwdShape<32> : Shape<2, 8> {};

// Pixel placement inside a tile.  Each wavefront owns a compact SUBW x SUBH
// block of the tile (8x8 for tile 8; 16 columns wide otherwise: 16x16 at 4 px/lane,
// 16x32 at 8 px/lane); lane l owns column l % SUBW of that block and rows
// l / SUBW + p * RS, p < PPL (RS = SUBH / PPL).  Pixel slot p of the wave is then
// the band of rows [p RS, (p + 1) RS) of the block, so a splat that misses a band
// is skipped by the whole wave for that slot.
template <int TILE, class SHAPE>
struct PixMap {
  static constexpr int WAVES = SHAPE::WAVES, PPL = SHAPE::PPL, NT = SHAPE::THREADS;
  static constexpr int SUBW = TILE < 16 ? TILE : 16, SUBH = 64 * PPL / SUBW;
  static_assert((TILE / SUBW) * (TILE / SUBH) == WAVES && SUBW * SUBH == 64 * PPL, "tile shape");
  static constexpr int WX = TILE / SUBW, WY = TILE / SUBH;  // wave blocks per tile row / column
  static constexpr int RS = SUBH / PPL;                      // row stride between a lane's pixels
  int v, x, y0, W, H, pix_off, tile;
  int tx0, ty0;  // top-left pixel of the tile
  int tcx, tcy;  // the tile's column and row in its view's grid
  int wx0, wy0;  // top-left pixel of this wave's block
  __device__ PixMap(const ViewTable& vt, int gt) {
    tile = gt;
    v = view_of_tile(vt, gt);
    const ViewGeom& g = vt.v[v];
    W = g.W;
    H = g.H;
    pix_off = g.pix_off;
    const int lt = gt - g.tile_off;
    const int tx = lt % g.TX, ty = lt / g.TX;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    tcx = tx;
    tcy = ty;
    tx0 = tx * TILE;
    ty0 = ty * TILE;
    wx0 = tx0 + (w % WX) * SUBW;
    wy0 = ty0 + (w / WX) * SUBH;
    x = wx0 + lane % SUBW;
    y0 = wy0 + lane / SUBW;
  }
  __device__ int row(int p) const { return y0 + p * RS; }
  __device__ bool inside(int p) const { return x < W && row(p) < H; }
  __device__ int pix(int p) const { return pix_off + row(p) * W + x; }
  __device__ int chan(int p, int c) const { return 3 * pix_off + c * W * H + row(p) * W + x; }
};

// Wave-level cull of a splat.  A pixel evaluates q = d^T Q d (d = pixel - mean, Q = [[a,b],[b,c]] the conic)
// in FP32 as -2 power and passes the exponent test only where that value is at most thr = -2 cutoff.  For a
// positive-definite Q the minimum of q over the rectangle of a wavefront's pixel centres is found exactly with
// two clamped one-dimensional minimizations: it is 0 when the mean lies inside; otherwise it lies on the
// rectangle's edge that faces the mean along x or along y (any other boundary point p with q(p) > 0 has t p,
// t < 1, inside the rectangle and q(t p) = t^2 q(p) < q(p)).  Along the line x = X, q is the parabola
// c y^2 + 2 b X y + a X^2 with its minimum at y = -b X / c, clamped to the rectangle, and likewise along
// y = Y.  Evaluating the line x = clamp(0, x0, x1) and the line y = clamp(0, y0, y1) thus gives two values
// of q on the rectangle whose smaller is its minimum.  The test is in natural units (thr = -2 cutoff); the
// pixels evaluate log2(e) times the exponent against log2(e) times the cutoff.  The FP32 rounding of this
// test and of every pixel's own evaluation, the base-2 scaling included, is below 1e-6 of
// |a| dx^2 + 2|b dx dy| + |c| dy^2 (which is at least q, so at least thr near the ellipse, and so also covers
// the rounding of the scaled cutoff), bounded over the block by (a + |b|) DX^2 + (c + |b|) DY^2 (DX, DY the
// largest |dx|, |dy|); a block is skipped only when both values exceed thr by 4e-6 of that bound.  Every pixel
// of a skipped block then computes an exponent below its cutoff, so the cull changes no result.  A splat with opacity below alpha_min (1 - 1e-3) or NaN can never
// blend (its exponent is at most 0) and is listed nowhere; a conic not shown positive definite is listed for
// every block.
constexpr float kQErr = 4.0e-6f;
struct CullConic {
  float a, c, b2, nbia, nbic, ka, kc, thr;
  int mode;  // 0: test the blocks, 1: list nowhere, 2: list everywhere
};
__device__ __forceinline__ CullConic cull_conic(float ca, float cb, float cc, float opacity, float alpha_min,
                                                float thr) {
  CullConic k;
  const bool pd = ca > 0.0f && cc > 0.0f && ca * cc > (cb * cb) * 1.00001f;
  k.mode = !(opacity >= alpha_min * 0.999f) ? 1 : (pd ? 0 : 2);
  k.a = ca;
  k.c = cc;
  k.b2 = cb + cb;
  k.nbia = -cb * __builtin_amdgcn_rcpf(ca);
  k.nbic = -cb * __builtin_amdgcn_rcpf(cc);
  k.ka = kQErr * (ca + fabsf(cb));
  k.kc = kQErr * (cc + fabsf(cb));
  k.thr = thr;
  return k;
}

// The bins as the raster kernels read them: tile lists (ids, ranges) or
// window lists (items, win_ranges), as gs_bins documents them.
struct ListArgs {
  const uint32_t* ids;
  const uint2* ranges;
  const uint2* items;
  const uint32_t* win_ranges;
};

// A tile's run of list positions [s, e): of its own list, or (WIN) of its
// binning window's list, whose items it takes where their clipped rect covers
// the tile's position (lx, ly) in the window.  The window list is in the
// order of every tile's list, so the covering items are the tile's list.
struct TileRun {
  int s, e;
  uint32_t lx, ly;
};
template <bool WIN, class PM>
__device__ __forceinline__ TileRun tile_run(const ListArgs& la, const ViewTable& vt, const PM& pm) {
  TileRun tr;
  if constexpr (WIN) {
    const ViewGeom& g = vt.v[pm.v];
    const int w = g.win_off + (pm.tcy >> kWinShift) * g.WX + (pm.tcx >> kWinShift);
    tr.s = (int)la.win_ranges[w];
    tr.e = (int)la.win_ranges[vt.total_windows + w];
    tr.lx = (uint32_t)(pm.tcx & (kWinSide - 1));
    tr.ly = (uint32_t)(pm.tcy & (kWinSide - 1));
  } else {
    const uint2 rg = la.ranges[pm.tile];
    tr.s = (int)rg.x;
    tr.e = (int)rg.y;
    tr.lx = tr.ly = 0u;
  }
  return tr;
}

// Whether a window item's clipped rect (lx0 | lx1 << 4 | ly0 << 8 | ly1 << 12, half-open, lx0 < lx1 and
// ly0 < ly1) covers window tile (lx, ly): one unsigned comparison per axis.
__device__ __forceinline__ bool item_covers(uint32_t code, uint32_t lx, uint32_t ly) {
  const uint32_t x0 = code & 15u, x1 = (code >> 4) & 15u, y0 = (code >> 8) & 15u, y1 = (code >> 12) & 15u;
  return (lx - x0) < (x1 - x0) && (ly - y0) < (y1 - y0);
}

// One splat record loaded into registers ahead of its batch (prefetch): list
// position idx of the tile's run; `valid` when it is an entry of the tile.
struct SplatLoader {
  float4 a, b, c;  // record words 0-3, 4-7, 8-11
  uint32_t id;
  bool valid;
  template <bool WIN>
  __device__ __forceinline__ void fetch(const float* __restrict__ rec, const ListArgs& la, const TileRun& tr,
                                        int idx) {
    valid = idx >= tr.s && idx < tr.e;
    if (valid) {
      if constexpr (WIN) {
        // one 8-byte load (pair and clipped rect together), then the cover test
        const unsigned long long it = reinterpret_cast<const unsigned long long*>(la.items)[idx];
        id = (uint32_t)it;
        valid = item_covers((uint32_t)(it >> 32), tr.lx, tr.ly);
      } else {
        id = la.ids[idx];
      }
    }
    if (valid) {
      const float4* r = reinterpret_cast<const float4*>(rec + (size_t)id * GS_REC_FLOATS);
      a = r[0];
      b = r[1];
      c = r[2];
    }
  }
};

// The pixel blocks of a tile's wavefronts (pixel centres inside the image),
// as WX column ranges and WY row ranges; a block entirely outside the image
// has hi < lo.
template <class PM>
struct BlockBoxes {
  float x_lo[PM::WX], x_hi[PM::WX], y_lo[PM::WY], y_hi[PM::WY];
  int all;  // bit w: wavefront w's block holds a pixel of the image
  __device__ explicit BlockBoxes(const PM& pm) {
    // tile-level values, the same in every lane: scalar registers
    const int tx0 = __builtin_amdgcn_readfirstlane(pm.tx0), ty0 = __builtin_amdgcn_readfirstlane(pm.ty0);
    const int W = __builtin_amdgcn_readfirstlane(pm.W), H = __builtin_amdgcn_readfirstlane(pm.H);
#pragma unroll
    for (int c = 0; c < PM::WX; ++c) {
      x_lo[c] = (float)(tx0 + c * PM::SUBW);
      x_hi[c] = (float)(min(tx0 + (c + 1) * PM::SUBW, W) - 1);
    }
#pragma unroll
    for (int r = 0; r < PM::WY; ++r) {
      y_lo[r] = (float)(ty0 + r * PM::SUBH);
      y_hi[r] = (float)(min(ty0 + (r + 1) * PM::SUBH, H) - 1);
    }
    all = 0;
#pragma unroll
    for (int r = 0; r < PM::WY; ++r)
#pragma unroll
      for (int c = 0; c < PM::WX; ++c)
        if (x_lo[c] <= x_hi[c] && y_lo[r] <= y_hi[r]) all |= 1 << (r * PM::WX + c);
  }
  // Bit w set: a pixel of wavefront w's block may pass the exponent test of the splat at (mx, my).
  __device__ __forceinline__ int mask(float mx, float my, const CullConic& k) const {
    float x0[PM::WX], x1[PM::WX], axx[PM::WX], bx2[PM::WX], tx[PM::WX], lx[PM::WX];
    float y0[PM::WY], y1[PM::WY], cyy[PM::WY], by2[PM::WY], ty[PM::WY], ly[PM::WY];
#pragma unroll
    for (int c = 0; c < PM::WX; ++c) {
      x0[c] = x_lo[c] - mx;
      x1[c] = x_hi[c] - mx;
      const float xn = __builtin_amdgcn_fmed3f(0.0f, x0[c], x1[c]);
      axx[c] = (k.a * xn) * xn;
      bx2[c] = k.b2 * xn;
      tx[c] = k.nbic * xn;
      const float dx = fmaxf(fabsf(x0[c]), fabsf(x1[c]));
      lx[c] = fmaf(k.ka * dx, dx, k.thr);
    }
#pragma unroll
    for (int r = 0; r < PM::WY; ++r) {
      y0[r] = y_lo[r] - my;
      y1[r] = y_hi[r] - my;
      const float yn = __builtin_amdgcn_fmed3f(0.0f, y0[r], y1[r]);
      cyy[r] = (k.c * yn) * yn;
      by2[r] = k.b2 * yn;
      ty[r] = k.nbia * yn;
      const float dy = fmaxf(fabsf(y0[r]), fabsf(y1[r]));
      ly[r] = (k.kc * dy) * dy;
    }
    int m = 0;
#pragma unroll
    for (int r = 0; r < PM::WY; ++r)
#pragma unroll
      for (int c = 0; c < PM::WX; ++c) {
        const float ys = __builtin_amdgcn_fmed3f(tx[c], y0[r], y1[r]);
        const float qv = fmaf(fmaf(k.c, ys, bx2[c]), ys, axx[c]);
        const float xs = __builtin_amdgcn_fmed3f(ty[r], x0[c], x1[c]);
        const float qh = fmaf(fmaf(k.a, xs, by2[r]), xs, cyy[r]);
        const float lim = lx[c] + ly[r];
        if (!(qv > lim) || !(qh > lim)) m |= 1 << (r * PM::WX + c);
      }
    m = k.mode == 0 ? m : (k.mode == 2 ? all : 0);
    return m & all;
  }
};

// LDS of one batch of RPL records per lane (RPL x NT entries): what the pixel
// loop reads per entry, and per wavefront the ordered list of the batch entries
// its pixel block can see.  Entry r NT + t of the batch is record r of thread t.
// RANK: also each valid entry's rank among the batch's valid entries (its
// position in the tile's list relative to the batch's first entry of the tile).
template <class PM, int RPL, bool RANK = false>
struct BatchLds {
  static constexpr int NB = RPL * PM::NT;
  float4 a[NB];  // (mean x, mean y, a'/2, b') for the conic (a, b, c), ' = times log2(e)
  float4 b[NB];  // (c'/2, opacity, qmax (the exponent cutoff as a bound on q), r)
  float4 c[NB];  // (g, b, unused, unused): 16-byte rows, so one index scale serves all three arrays
  uint32_t id[NB];
  uint16_t list[PM::WAVES][NB];
  int cnt[RPL][PM::WAVES][PM::WAVES];  // [record][staging wave][listing wave]
  uint16_t rank[RANK ? NB : 1];
  int vcnt[RANK ? RPL : 1][PM::WAVES];  // valid entries per [record][staging wave]
};

// Stages the batch held by `ld` (RPL entries per thread): entry data into LDS,
// the cull of every wavefront block done once here per entry, and each
// wavefront's list built in entry order (ballots, then the staging waves'
// counts in order, record by record).  Ends with a barrier; returns the
// calling wave's count.
template <class PM, int RPL, bool RANK = false>
__device__ __forceinline__ int stage_batch(const SplatLoader (&ld)[RPL], const BlockBoxes<PM>& bx, float alpha_min,
                                           BatchLds<PM, RPL, RANK>& L, bool with_id, int* n_valid = nullptr) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int mask[RPL];
  uint64_t bal[RPL][PM::WAVES];
  uint64_t vb[RANK ? RPL : 1];
  if constexpr (RANK) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      vb[r] = __ballot(ld[r].valid);
      if (lane == 0) L.vcnt[r][w] = (int)__popcll(vb[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int slot = r * PM::NT + t;
    mask[r] = 0;
    if (ld[r].valid) {
      const SplatLoader& d = ld[r];
      const float cut = power_cutoff(d.b.y, alpha_min);
      mask[r] = bx.mask(d.a.x, d.a.y, cull_conic(d.a.z, d.a.w, d.b.x, d.b.y, alpha_min, -2.0f * cut));
      L.a[slot] = make_float4(d.a.x, d.a.y, (0.5f * kLog2e) * d.a.z, kLog2e * d.a.w);
      L.b[slot] = make_float4((0.5f * kLog2e) * d.b.x, d.b.y, fmaxf(-kLog2e * cut, 0.0f), d.b.z);
      L.c[slot] = make_float4(d.b.w, d.c.x, 0.0f, 0.0f);
      if (with_id) L.id[slot] = d.id;
    }
#pragma unroll
    for (int q = 0; q < PM::WAVES; ++q) bal[r][q] = __ballot((mask[r] >> q) & 1);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < PM::WAVES; ++q) L.cnt[r][w][q] = (int)__popcll(bal[r][q]);
    }
  }
  __syncthreads();
  if constexpr (RANK) {
    // slot r NT + t is list position (valid slots of earlier records and earlier waves) + (lanes below)
    int before = 0, total = 0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      int here = before;
#pragma unroll
      for (int w2 = 0; w2 < PM::WAVES; ++w2) {
        const int c = L.vcnt[r][w2];
        here += w2 < w ? c : 0;
        before += c;
      }
      if (ld[r].valid) L.rank[r * PM::NT + t] = (uint16_t)(here + (int)__popcll(vb[r] & lt));
    }
    total = before;
    *n_valid = total;
  }
  int mine = 0;
#pragma unroll
  for (int q = 0; q < PM::WAVES; ++q) {
    int off = 0;  // the entries of earlier records, then of earlier staging waves of this record
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      int here = off;
#pragma unroll
      for (int w2 = 0; w2 < PM::WAVES; ++w2) {
        const int c = L.cnt[r][w2][q];
        here += w2 < w ? c : 0;
        off += c;
      }
      if ((mask[r] >> q) & 1) L.list[q][here + (int)__popcll(bal[r][q] & lt)] = (uint16_t)(r * PM::NT + t);
    }
    mine = q == w ? off : mine;
  }
  __syncthreads();
  return mine;
}

// ---------------------------------------------------------------------------
// Forward.
// ---------------------------------------------------------------------------
// A pixel that has stopped gets row coordinate +inf: its q is then +inf or
// NaN and fails the range test, so no separate flag is tested.
// STATE: the pixel state (T_final, n_contrib) is written (not under the checkpoint flag).
// (six wavefronts per SIMD: measured faster than five, despite a few bytes of spill outside the loop;
// at tile 32 with two records per lane the batch's LDS leaves room for four)
// RPL: splat records each lane stages per LDS batch.  WIN: the bins are window lists.
template <int TILE, bool STATE, int RPL, bool WIN>
__global__ __launch_bounds__(FwdShape<TILE>::THREADS)
__attribute__((amdgpu_waves_per_eu(TILE == 32 && RPL == 2 ? 4 : 6))) void k_render_fwd(
    ViewTable vt, const float* __restrict__ rec, ListArgs la, RasterConsts rc, float* __restrict__ img,
    float* __restrict__ tfin, int32_t* __restrict__ ncon, const float* __restrict__ target,
    float* __restrict__ tile_loss) {
  using PM = PixMap<TILE, FwdShape<TILE>>;
  constexpr int PPL = PM::PPL, NT = PM::NT;
  constexpr int NB = RPL * NT;  // entries per batch
  constexpr bool RANK = WIN && STATE;  // list positions of window-list entries (for n_contrib)
  __shared__ BatchLds<PM, RPL, RANK> L;
  __shared__ float s_loss[PM::WAVES];
  const PM pm(vt, blockIdx.x);
  const float amax = __builtin_canonicalizef(rc.alpha_max);  // canonical once: fminf needs no per-use quieting
  const BlockBoxes<PM> boxes(pm);
  const int w = threadIdx.x >> 6;
  float T[PPL], C[PPL][3], fy[PPL];
  int last[PPL];
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    T[p] = 1.0f;
    C[p][0] = C[p][1] = C[p][2] = 0.0f;
    last[p] = 0;
    fy[p] = pm.inside(p) ? (float)pm.row(p) : INFINITY;
  }
  const TileRun tr = tile_run<WIN>(la, vt, pm);
  const int s = tr.s, e = tr.e;
  const float fx = (float)pm.x;
  int vbase = 0;  // RANK: the tile's entries in earlier batches
  SplatLoader ld[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) ld[r].template fetch<WIN>(rec, la, tr, s + r * NT + (int)threadIdx.x);
  for (int base = s; base < e; base += NB) {
    int alive = 0;
#pragma unroll
    for (int p = 0; p < PPL; ++p) alive |= fy[p] != INFINITY ? 1 : 0;
    if (__syncthreads_count(alive) == 0) break;
    int n_valid = 0;
    const int n = stage_batch<PM, RPL, RANK>(ld, boxes, rc.alpha_min, L, false, &n_valid);
#pragma unroll
    for (int r = 0; r < RPL; ++r)  // next batch, in flight during this one
      ld[r].template fetch<WIN>(rec, la, tr, base + NB + r * NT + (int)threadIdx.x);
    // a wavefront whose pixels have all stopped only keeps the block's barriers
    // (wave-uniform: kept in a scalar register, so the walk's loop control is scalar)
    const int cnt = __builtin_amdgcn_readfirstlane(__ballot(alive) != 0ull ? n : 0);
    for (int k = 0; k < cnt; ++k) {
      const int j = L.list[w][k];
      const float4 A = L.a[j];
      const float4 Bv = L.b[j];
      const float2 Cv = make_float2(L.c[j].x, L.c[j].y);
      const RowTerms rt = row_terms(fx - A.x, A.z, A.w);
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        const float q = splat_q(rt, Bv.x, fy[p] - A.y);
        // only an exponent in [cutoff, 0] can reach alpha_min; the wave skips a pixel slot no lane reaches
        if (!q_in_range(q, Bv.z)) continue;
        // the rest is branch-free: a pixel that does not blend gets weight 0, which adds exactly nothing
        const float oG = Bv.y * __builtin_amdgcn_exp2f(-q);
        const float alpha = fminf(oG, amax);  // one v_min (NaN, not reachable here, would give alpha_max)
        const float test = T[p] * (1.0f - alpha);
        const bool keep = alpha >= rc.alpha_min;
        const bool stop = keep && test < rc.t_min;
        const bool blend = keep && !stop;
        fy[p] = stop ? INFINITY : fy[p];
        const float wgt = blend ? alpha * T[p] : 0.0f;
        C[p][0] = fmaf(Bv.w, wgt, C[p][0]);
        C[p][1] = fmaf(Cv.x, wgt, C[p][1]);
        C[p][2] = fmaf(Cv.y, wgt, C[p][2]);
        T[p] = blend ? test : T[p];
        if (STATE) last[p] = blend ? (RANK ? vbase + (int)L.rank[j] : base - s + j) + 1 : last[p];
      }
    }
    vbase += n_valid;
  }
  float lsum = 0.0f;
  float tg[PPL][3];  // the target's pixels, all loads in flight before the stores
  if (target) {
#pragma unroll
    for (int p = 0; p < PPL; ++p)
#pragma unroll
      for (int c = 0; c < 3; ++c) tg[p][c] = target[pm.inside(p) ? pm.chan(p, c) : 0];
  }
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    if (!pm.inside(p)) continue;
    const float out[3] = {C[p][0] + T[p] * rc.bg0, C[p][1] + T[p] * rc.bg1, C[p][2] + T[p] * rc.bg2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      img[pm.chan(p, c)] = out[c];
      if (target) lsum += fabsf(out[c] - tg[p][c]);
    }
    if (STATE) {
      tfin[pm.pix(p)] = T[p];
      ncon[pm.pix(p)] = last[p];
    }
  }
  if (tile_loss) {
    lsum = wave_sum(lsum);
    if ((threadIdx.x & 63) == 0) s_loss[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.0f;
      for (int q = 0; q < PM::WAVES; ++q) t += s_loss[q];
      tile_loss[blockIdx.x] = t;
    }
  }
}

// Per-view L1 term from the per-tile partial sums (fixed order).
__global__ __launch_bounds__(256) void k_loss_reduce(ViewTable vt, const float* __restrict__ tile_loss,
                                                     float* __restrict__ loss_out) {
  __shared__ float s_w[4];
  const ViewGeom& g = vt.v[blockIdx.x];
  const int nt = g.TX * g.TY;
  float acc = 0.0f;
  for (int t = threadIdx.x; t < nt; t += 256) acc += tile_loss[g.tile_off + t];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) loss_out[blockIdx.x] = (s_w[0] + s_w[1] + s_w[2] + s_w[3]) / (3.0f * (float)g.W * (float)g.H);
}

// ---------------------------------------------------------------------------
// Backward.
//
// Per entry the wavefront needs, besides the colour terms, the moments of
// u = dL/dpower over its pixels: Sx = sum u dx, Sy = sum u dy, Sxx = sum u dx^2,
// Sxy = sum u dx dy, Syy = sum u dy^2.  The image-space gradients follow
// exactly, since the conic is constant per entry: dL/dmean = (a Sx + b Sy,
// b Sx + c Sy), dL/d(a, b, c) = (-Sxx/2, -Sxy, -Syy/2).  A lane's pixels share
// one column, so dx is the same for all of them: the lane sums only U = sum u,
// Uy = sum u dy and Uyy = sum u dy^2 over its pixels, and its moments are
// dx U, Uy, dx^2 U, dx Uy, Uyy.  U is also the opacity term: where alpha is not
// clamped, u = dL/dalpha alpha = o dL/dalpha G, so dL/do = U / o.  The 9 sums are reduced over the
// wavefront by a reduce-scatter: each permlane32/permlane16 swap adds two
// different values at once (one per half of the exchanged lanes), leaving
// three registers whose 16-lane rows each hold one partial sum, which DPP row
// operations complete.
// ---------------------------------------------------------------------------
struct Acc9 {
  float sx, sxx, sxy, syy, r, g, b, o, sy;
};
// A lane's sums over its pixels for the current entry.
struct Acc6 {
  float r, g, b, u, uy, uyy;
};
struct Red3 {
  float k0, k1, k2;
};

__device__ __forceinline__ float swap_add32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_add16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float row_sum(float x) {
  x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp<0x141>(x);  // row_half_mirror
  return x + dpp<0x140>(x);  // row_mirror
}
// Needs all 64 lanes active.  k0 rows hold {sx, sxx, sxy, syy}, k1 rows
// {r, g, b, o}, k2 holds sy in every row; which row holds which value is
// found once per kernel (wave_roles) rather than assumed.
__device__ __forceinline__ Red3 reduce_scatter(const Acc9& a) {
  const float h0 = swap_add32(a.sx, a.sxx), h1 = swap_add32(a.sxy, a.syy);
  const float h2 = swap_add32(a.r, a.g), h3 = swap_add32(a.b, a.o);
  const float h4 = swap_add32(a.sy, a.sy);
  return Red3{row_sum(swap_add16(h0, h1)), row_sum(swap_add16(h2, h3)), row_sum(swap_add16(h4, h4))};
}

// What this lane writes after a reduction: gradient component `comp` (-1:
// none) = ka * k0 + kc * k2 + k1c * k1, with (ka, kc) = (a, b) for the mean x
// term, (b, c) for mean y, else (k0c, 0); for the opacity k1c is 1 / opacity
// (the lanes sum dL/dalpha alpha, which is opacity times dL/dalpha G).
struct LaneRole {
  int comp;
  bool mean_x, mean_y, opacity;
  float k0c, k1c;
};
__device__ LaneRole wave_roles(int lane) {
  // one-hot tags 1..9 from lane 0 land, fully reduced, where the values do
  const float one = lane == 0 ? 1.0f : 0.0f;
  const Red3 t = reduce_scatter(Acc9{1 * one, 2 * one, 3 * one, 4 * one, 5 * one, 6 * one, 7 * one, 8 * one, 9 * one});
  const int t0 = (int)(t.k0 + 0.5f), t1 = (int)(t.k1 + 0.5f);
  const int r16 = lane & 15;
  LaneRole rl{-1, false, false, false, 0.0f, 0.0f};
  if (t0 == 1 && r16 == 0) { rl.comp = 0; rl.mean_x = true; }
  else if (t0 == 1 && r16 == 1) { rl.comp = 1; rl.mean_y = true; }
  else if (t0 == 2 && r16 == 0) { rl.comp = 2; rl.k0c = -0.5f; }
  else if (t0 == 3 && r16 == 0) { rl.comp = 3; rl.k0c = -1.0f; }
  else if (t0 == 4 && r16 == 0) { rl.comp = 4; rl.k0c = -0.5f; }
  else if (r16 == 2 && t1 >= 5 && t1 <= 8) {  // o -> 5, r,g,b -> 6,7,8
    rl.comp = t1 == 8 ? 5 : t1 + 1;
    rl.opacity = t1 == 8;
    rl.k1c = 1.0f;
  }
  return rl;
}

// Per-lane sums of the homodirectional (AbsGS) view-space gradient: the
// magnitudes of each pixel's two mean components, |u (a dx + b dy)| and
// |u (b dx + c dy)|, which the moments above cannot give.  Reduced like sy: a
// swap between the wave halves puts one value's partials in each half, the
// row swap and row sum complete them; which lane writes which component is
// found once per kernel from one-hot tags, one lane per component.
__device__ __forceinline__ float reduce_pair(float a, float b) {
  return row_sum(swap_add16(swap_add32(a, b), swap_add32(a, b)));
}
__device__ int abs_role(int lane) {
  const float one = lane == 0 ? 1.0f : 0.0f;
  const int t = (int)(reduce_pair(1.0f * one, 2.0f * one) + 0.5f);
  const unsigned long long m0 = __ballot(t == 1), m1 = __ballot(t == 2);
  if (m0 != 0ull && lane == __ffsll((long long)m0) - 1) return 0;
  if (m1 != 0ull && lane == __ffsll((long long)m1) - 1) return 1;
  return -1;
}

// One front-to-back sweep per pixel, with the forward's decisions: the colour
// behind entry k is S_k = C_pixel - sum_{m<=k} c_m alpha_m T_m (C_pixel the
// rendered value, background included), so neither the final transmittance
// nor the contributor count is needed and nothing is replayed or divided.
// Only its projection on dL/dC enters the gradient, so a pixel carries the
// scalar D_k = dL/dC . S_k, updated by the entry's dL/dC . c_k.
// With ABS the kernel also adds the homodirectional view-space gradient of
// each (view, Gaussian) pair into abs2d [V*N][2].
template <int TILE, bool ABS, int RPL, bool WIN>
// (five wavefronts per SIMD: 96 registers, no spill; measured 10% faster than four)
__global__ __launch_bounds__(BwdShape<TILE>::THREADS)
__attribute__((amdgpu_waves_per_eu(BwdShape<TILE>::PPL == 8 ? 4 : 5))) void k_render_bwd(
    ViewTable vt, const float* __restrict__ rec, ListArgs la, RasterConsts rc, const float* __restrict__ img,
    int loss_kind, const float* __restrict__ target, const float* __restrict__ dl_dimage,
    float* __restrict__ grad2d, float* __restrict__ abs2d) {
  using PM = PixMap<TILE, BwdShape<TILE>>;
  constexpr int PPL = PM::PPL, NT = PM::NT;
  constexpr int NB = RPL * NT;  // entries per batch
  __shared__ BatchLds<PM, RPL> L;
  const PM pm(vt, blockIdx.x);
  const float amax = __builtin_canonicalizef(rc.alpha_max);  // canonical once: fminf needs no per-use quieting
  const BlockBoxes<PM> boxes(pm);
  const TileRun tr = tile_run<WIN>(la, vt, pm);
  const int s = tr.s, e = tr.e;
  const float fx = (float)pm.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const LaneRole role = wave_roles(lane);
  const int arole = ABS ? abs_role(lane) : -1;
  // per pixel: transmittance in front of the current entry, dL/dC . (colour still behind it), dL/dC;
  // a pixel that has stopped gets row coordinate +inf (see k_render_fwd)
  float T[PPL], Dp[PPL], dl[PPL][3], fy[PPL];
  const float wv = 1.0f / (3.0f * (float)pm.W * (float)pm.H);
  {
    // every pixel's image and target (or dL/dimage) loads first, all in flight together (a pixel
    // outside the image reads element 0 and discards it)
    const bool l1 = loss_kind == GS_LOSS_L1;
    const float* __restrict__ second = l1 ? target : dl_dimage;
    float col[PPL][3], aux[PPL][3];
#pragma unroll
    for (int p = 0; p < PPL; ++p)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int at = pm.inside(p) ? pm.chan(p, c) : 0;
        col[p][c] = img[at];
        aux[p][c] = second[at];
      }
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const bool in = pm.inside(p);
      fy[p] = in ? (float)pm.row(p) : INFINITY;
      T[p] = 1.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float r = col[p][c] - aux[p][c];
        const float d = l1 ? (r > 0.0f ? wv : (r < 0.0f ? -wv : 0.0f)) : aux[p][c];
        dl[p][c] = in ? d : 0.0f;
        col[p][c] = in ? col[p][c] : 0.0f;
      }
      Dp[p] = fmaf(dl[p][2], col[p][2], fmaf(dl[p][1], col[p][1], dl[p][0] * col[p][0]));
    }
  }
  Acc6 acc{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  float amx = 0.0f, amy = 0.0f;  // ABS: the lane's sums of |dL_p/dmean| for the current entry
  SplatLoader ld[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) ld[r].template fetch<WIN>(rec, la, tr, s + r * NT + (int)threadIdx.x);
  for (int base = s; base < e; base += NB) {
    int alive = 0;
#pragma unroll
    for (int p = 0; p < PPL; ++p) alive |= fy[p] != INFINITY ? 1 : 0;
    if (__syncthreads_count(alive) == 0) break;
    const int n = stage_batch<PM, RPL>(ld, boxes, rc.alpha_min, L, true);
#pragma unroll
    for (int r = 0; r < RPL; ++r)  // next batch, in flight during this one
      ld[r].template fetch<WIN>(rec, la, tr, base + NB + r * NT + (int)threadIdx.x);
    // (wave-uniform: kept in a scalar register, so the walk's loop control is scalar)
    const int cnt = __builtin_amdgcn_readfirstlane(__ballot(alive) != 0ull ? n : 0);
    for (int k = 0; k < cnt; ++k) {
      const int j = L.list[w][k];
      const float4 A = L.a[j];
      const float4 Bv = L.b[j];
      const float2 Cv = make_float2(L.c[j].x, L.c[j].y);
      const float dx = fx - A.x;
      const RowTerms rt = row_terms(dx, A.z, A.w);
      // the natural conic (a, b, c) from the staged base-2 factors
      const float ca = (2.0f * kLn2) * A.z, cb = kLn2 * A.w, cc = (2.0f * kLn2) * Bv.x;
      const float tx = ABS ? ca * dx : 0.0f, ty = ABS ? cb * dx : 0.0f;
      bool any = false;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        const float dy = fy[p] - A.y;
        const float q = splat_q(rt, Bv.x, dy);
        // only an exponent in [cutoff, 0] can reach alpha_min; the wave skips a pixel slot no lane reaches
        if (!q_in_range(q, Bv.z)) continue;
        // the rest is branch-free: a pixel that does not blend gets weight 0 and no exponent
        // gradient, which add exactly nothing (every factor is finite: 1 - alpha >= 1 - alpha_max)
        const float oG = Bv.y * __builtin_amdgcn_exp2f(-q);
        const bool below = oG <= amax;
        const float alpha = fminf(oG, amax);  // one v_min, independent of the compare
        const float om = 1.0f - alpha;
        const float test = T[p] * om;
        const bool keep = alpha >= rc.alpha_min;
        const bool stop = keep && test < rc.t_min;
        const bool blend = keep && !stop;
        fy[p] = stop ? INFINITY : fy[p];
        any = any || blend;
        const float wgt = blend ? alpha * T[p] : 0.0f;
        acc.r = fmaf(dl[p][0], wgt, acc.r);
        acc.g = fmaf(dl[p][1], wgt, acc.g);
        acc.b = fmaf(dl[p][2], wgt, acc.b);
        const float dc = fmaf(dl[p][2], Cv.y, fmaf(dl[p][1], Cv.x, dl[p][0] * Bv.w));
        Dp[p] = fmaf(-dc, wgt, Dp[p]);  // now dL/dC . S_k, the colour behind this entry
        const float dLda = fmaf(T[p], dc, -Dp[p] * __builtin_amdgcn_rcpf(om));
        T[p] = blend ? test : T[p];
        const bool unclamped = blend && below;  // d alpha / d(o, power) = 0 where clamped
        const float dLdp = unclamped ? dLda * alpha : 0.0f;
        const float uy = dLdp * dy;
        acc.u += dLdp;
        acc.uy += uy;
        acc.uyy = fmaf(uy, dy, acc.uyy);
        if (ABS) {
          amx += fabsf(dLdp * fmaf(cb, dy, tx));
          amy += fabsf(dLdp * fmaf(cc, dy, ty));
        }
      }
      if (__ballot(any) != 0ull) {
        const float sx = dx * acc.u;
        const Red3 r = reduce_scatter(Acc9{sx, dx * sx, dx * acc.uy, acc.uyy, acc.r, acc.g, acc.b, acc.u, acc.uy});
        const float ka = role.mean_x ? ca : (role.mean_y ? cb : role.k0c);
        const float kc = role.mean_x ? cb : (role.mean_y ? cc : 0.0f);
        const float k1 = role.opacity ? __builtin_amdgcn_rcpf(Bv.y) : role.k1c;  // a blended entry has opacity >= alpha_min
        const float val = fmaf(ka, r.k0, fmaf(kc, r.k2, k1 * r.k1));
        if (role.comp >= 0) atomicAdd(grad2d + (size_t)L.id[j] * GS_GRAD2D_FLOATS + role.comp, val);
        acc = Acc6{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (ABS) {
          const float t = reduce_pair(amx, amy);
          if (arole >= 0) atomicAdd(abs2d + (size_t)L.id[j] * 2 + arole, t);
          amx = amy = 0.0f;
        }
      }
    }
  }
}

// Work counts of the per-pixel blending as defined (no cull, no exponent
// cutoff): per pixel, the list entries evaluated until it stops (list end, or
// the entry that would take T below t_min, inclusive), the entries blended,
// and n_contrib; summed over the image into out[0..2] (one 64-bit atomic per
// wavefront and count).
template <int TILE, bool WIN>
__global__ __launch_bounds__(FwdShape<TILE>::THREADS) void k_render_stats(
    ViewTable vt, const float* __restrict__ rec, ListArgs la, RasterConsts rc, unsigned long long* __restrict__ out) {
  using PM = PixMap<TILE, FwdShape<TILE>>;
  constexpr int PPL = PM::PPL, NT = PM::NT;
  __shared__ float4 s_a[NT];  // (mean x, mean y, a'/2, b'), ' = times log2(e)
  __shared__ float2 s_b[NT];  // (c'/2, opacity)
  __shared__ int s_wc[PM::WAVES];  // WIN: the tile's entries per wavefront of the batch
  const PM pm(vt, blockIdx.x);
  const float amax = __builtin_canonicalizef(rc.alpha_max);  // canonical once: fminf needs no per-use quieting
  float T[PPL], fy[PPL];
  int last[PPL], evals[PPL], blended[PPL];
  bool done[PPL];
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    T[p] = 1.0f;
    last[p] = evals[p] = blended[p] = 0;
    done[p] = !pm.inside(p);
    fy[p] = (float)pm.row(p);
  }
  const TileRun tr = tile_run<WIN>(la, vt, pm);
  const int s = tr.s, e = tr.e;
  const float fx = (float)pm.x;
  int vbase = 0;  // the tile's entries in earlier batches
  SplatLoader ld;
  for (int base = s; base < e; base += NT) {
    int alive = 0;
#pragma unroll
    for (int p = 0; p < PPL; ++p) alive |= done[p] ? 0 : 1;
    if (__syncthreads_count(alive) == 0) break;
    ld.template fetch<WIN>(rec, la, tr, base + (int)threadIdx.x);
    int slot = (int)threadIdx.x, cnt = min(NT, e - base);
    if constexpr (WIN) {
      // the batch's entries of the tile, packed in list order
      const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
      const uint64_t b = __ballot(ld.valid);
      if (lane == 0) s_wc[w] = (int)__popcll(b);
      __syncthreads();
      int before = 0;
      cnt = 0;
#pragma unroll
      for (int q = 0; q < PM::WAVES; ++q) {
        before += q < w ? s_wc[q] : 0;
        cnt += s_wc[q];
      }
      slot = before + (int)__popcll(b & (lane == 0 ? 0ull : (~0ull >> (64 - lane))));
    }
    if (ld.valid) {
      s_a[slot] = make_float4(ld.a.x, ld.a.y, (0.5f * kLog2e) * ld.a.z, kLog2e * ld.a.w);
      s_b[slot] = make_float2((0.5f * kLog2e) * ld.b.x, ld.b.y);
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 cu = s_a[j];
      const float2 geo = s_b[j];
      const RowTerms rt = row_terms(fx - cu.x, cu.z, cu.w);
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        if (done[p]) continue;
        ++evals[p];
        const float q = splat_q(rt, geo.x, fy[p] - cu.y);
        if (q < 0.0f) continue;  // power > 0
        const float oG = geo.y * __builtin_amdgcn_exp2f(-q);
        const float alpha = fminf(oG, amax);  // one v_min (NaN, not reachable here, would give alpha_max)
        if (!(alpha >= rc.alpha_min)) continue;
        const float test = T[p] * (1.0f - alpha);
        if (test < rc.t_min) {
          done[p] = true;
          continue;
        }
        T[p] = test;
        ++blended[p];
        last[p] = (WIN ? vbase : base - s) + j + 1;
      }
    }
    __syncthreads();
    vbase += cnt;
  }
  unsigned long long c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    c0 += (unsigned long long)evals[p];
    c1 += (unsigned long long)blended[p];
    c2 += (unsigned long long)last[p];
  }
  for (int o = 32; o > 0; o >>= 1) {
    c0 += __shfl_xor(c0, o);
    c1 += __shfl_xor(c1, o);
    c2 += __shfl_xor(c2, o);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(out, c0);
    atomicAdd(out + 1, c1);
    atomicAdd(out + 2, c2);
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void k_fill_f32(float* __restrict__ p, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

static RasterConsts consts_of(const gs_options* o) {
  return RasterConsts{o->alpha_min, o->alpha_max, o->t_min, o->bg[0], o->bg[1], o->bg[2], o->radius_sigmas};
}

static gs_status validate_raster_common(const gs_projected* proj, const gs_bins* bins, const gs_camera* cams,
                                        int32_t n_views, const gs_options* opts) {
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if (!proj || !proj->rec) return fail(GS_ERR_INVALID_VALUE, "proj->rec is NULL");
  if (!bins) return fail(GS_ERR_INVALID_VALUE, "bins is NULL");
  if (reinterpret_cast<uintptr_t>(proj->rec) % 16 != 0) return fail(GS_ERR_INVALID_VALUE, "rec must be 16-byte aligned");
  if (opts->flags & GS_OPT_WINDOW_LISTS) {
    if (!bins->items || !bins->win_ranges) return fail(GS_ERR_INVALID_VALUE, "bins->items/win_ranges is NULL");
    if (reinterpret_cast<uintptr_t>(bins->items) % 8 != 0)
      return fail(GS_ERR_INVALID_VALUE, "items must be 8-byte aligned");
  } else {
    if (!bins->ids || !bins->ranges) return fail(GS_ERR_INVALID_VALUE, "bins->ids/ranges is NULL");
    if (reinterpret_cast<uintptr_t>(bins->ranges) % 8 != 0)
      return fail(GS_ERR_INVALID_VALUE, "ranges must be 8-byte aligned");
  }
  return GS_OK;
}

static ListArgs list_args(const gs_bins* bins) {
  return ListArgs{bins->ids, reinterpret_cast<const uint2*>(bins->ranges), reinterpret_cast<const uint2*>(bins->items),
                  bins->win_ranges};
}

}  // namespace gs

extern "C" gs_status gs_render_fwd_workspace_size(const gs_camera* cams, int32_t n_views, const gs_options* opts,
                                                  size_t* bytes) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if (!bytes) return fail(GS_ERR_INVALID_VALUE, "bytes is NULL");
  *bytes = align256(sizeof(float) * (size_t)make_view_table(cams, n_views, opts->tile_size).total_tiles);
  return GS_OK;
}

extern "C" gs_status gs_render_bwd_workspace_size(int64_t n, int32_t n_views, size_t* bytes) {
  using namespace gs;
  if (!bytes) return fail(GS_ERR_INVALID_VALUE, "bytes is NULL");
  if (n < 1 || n_views < 1 || n_views > GS_MAX_VIEWS) return fail(GS_ERR_INVALID_VALUE, "bad n or n_views");
  *bytes = align256(sizeof(float) * GS_GRAD2D_FLOATS * (size_t)n * (size_t)n_views);
  return GS_OK;
}

namespace gs {

// The forward behind gs_render_fwd and gs_render_fwd_noalloc: `tile_loss` (total_tiles floats, or
// NULL when no loss value is requested) receives the per-tile L1 partial sums.
static gs_status render_fwd_impl(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_camera* cams,
                                 int32_t n_views, const gs_options* opts, const gs_loss* loss, const gs_image* out,
                                 const ViewTable& vt, float* tile_loss, hipStream_t st) {
  const bool want_loss = tile_loss != nullptr;
  const RasterConsts rc = consts_of(opts);
  const float* tgt = want_loss ? loss->target : nullptr;
  float* tf = opts->checkpoint ? nullptr : out->t_final;
  int32_t* nc = opts->checkpoint ? nullptr : out->n_contrib;
  const dim3 grid((unsigned)vt.total_tiles);
  const ListArgs la = list_args(bins);
  const bool win = (opts->flags & GS_OPT_WINDOW_LISTS) != 0;
  (void)n;
#define GS_LAUNCH_FWD_W(TILE_, NT_, RPL_, WIN_)                                                                 \
  do {                                                                                                         \
    if (tf)                                                                                                    \
      hipLaunchKernelGGL((k_render_fwd<TILE_, true, RPL_, WIN_>), grid, dim3(NT_), 0, st, vt, proj->rec, la, rc, \
                         out->rgb, tf, nc, tgt, tile_loss);                                                   \
    else                                                                                                       \
      hipLaunchKernelGGL((k_render_fwd<TILE_, false, RPL_, WIN_>), grid, dim3(NT_), 0, st, vt, proj->rec, la,    \
                         rc, out->rgb, tf, nc, tgt, tile_loss);                                               \
  } while (0)
#define GS_LAUNCH_FWD_R(TILE_, NT_, RPL_)           \
  do {                                             \
    if (win)                                       \
      GS_LAUNCH_FWD_W(TILE_, NT_, RPL_, true);     \
    else                                           \
      GS_LAUNCH_FWD_W(TILE_, NT_, RPL_, false);    \
  } while (0)
#define GS_LAUNCH_FWD(TILE_, NT_)                  \
  do {                                            \
    if (opts->lds_batch == 2)                     \
      GS_LAUNCH_FWD_R(TILE_, NT_, 2);             \
    else                                          \
      GS_LAUNCH_FWD_R(TILE_, NT_, 1);             \
  } while (0)
  switch (opts->tile_size) {
    case 8: GS_LAUNCH_FWD(8, FwdShape<8>::THREADS); break;
    case 16: GS_LAUNCH_FWD(16, FwdShape<16>::THREADS); break;
    default: GS_LAUNCH_FWD(32, FwdShape<32>::THREADS); break;
  }
#undef GS_LAUNCH_FWD_W
#undef GS_LAUNCH_FWD_R
#undef GS_LAUNCH_FWD
  if (want_loss) hipLaunchKernelGGL(k_loss_reduce, dim3(n_views), dim3(256), 0, st, vt, tile_loss, loss->loss_out);
  return check_launch("render forward");
}

// Validation shared by both forward entry points; *want_loss tells whether a loss value is requested.
static gs_status validate_render_fwd(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_camera* cams,
                                     int32_t n_views, const gs_options* opts, const gs_loss* loss,
                                     const gs_image* out, bool* want_loss) {
  gs_status s;
  if ((s = validate_raster_common(proj, bins, cams, n_views, opts)) != GS_OK) return s;
  if (n < 1) return fail(GS_ERR_INVALID_VALUE, "n must be >= 1");
  if (!out || !out->rgb) return fail(GS_ERR_INVALID_VALUE, "out->rgb is NULL");
  if (!opts->checkpoint && (!out->t_final || !out->n_contrib))
    return fail(GS_ERR_INVALID_VALUE, "t_final/n_contrib are required unless checkpoint is set");
  if (loss && loss->kind != GS_LOSS_NONE && loss->kind != GS_LOSS_L1 && loss->kind != GS_LOSS_EXTERNAL)
    return fail(GS_ERR_INVALID_VALUE, "unknown loss kind");
  *want_loss = loss && loss->kind == GS_LOSS_L1 && loss->loss_out;
  if (*want_loss && !loss->target) return fail(GS_ERR_INVALID_VALUE, "L1 loss needs a target");
  return GS_OK;
}

// Per-tile L1 partial sums of gs_render_fwd_noalloc: one array per GPU, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is not a device address): it
// takes the address hipGetSymbolAddress gives for the current device, once per device.
constexpr int64_t kNoAllocTiles = GS_NOALLOC_MAX_TILES;
static __device__ __align__(256) float scratch[kNoAllocTiles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kMaxDevices];

static gs_status noalloc_scratch(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

}  // namespace gs

extern "C" gs_status gs_render_fwd(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_camera* cams,
                                   int32_t n_views, const gs_options* opts, const gs_loss* loss, const gs_image* out,
                                   void* workspace, size_t workspace_bytes, void* stream) {
  using namespace gs;
  gs_status s;
  bool want_loss = false;
  if ((s = validate_render_fwd(proj, n, bins, cams, n_views, opts, loss, out, &want_loss)) != GS_OK) return s;
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  const size_t need = align256(sizeof(float) * (size_t)vt.total_tiles);
  if (want_loss && (!workspace || workspace_bytes < need))
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(need) + " bytes");
  return render_fwd_impl(proj, n, bins, cams, n_views, opts, loss, out, vt,
                         want_loss ? static_cast<float*>(workspace) : nullptr, as_stream(stream));
}

extern "C" gs_status gs_render_fwd_noalloc(const gs_projected* proj, int64_t n, const gs_bins* bins,
                                           const gs_camera* cams, int32_t n_views, const gs_options* opts,
                                           const gs_loss* loss, const gs_image* out, void* stream) {
  using namespace gs;
  gs_status s;
  bool want_loss = false;
  if ((s = validate_render_fwd(proj, n, bins, cams, n_views, opts, loss, out, &want_loss)) != GS_OK) return s;
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  if (want_loss && (int64_t)vt.total_tiles > kNoAllocTiles)
    return fail(GS_ERR_CAPACITY, "gs_render_fwd_noalloc: " + std::to_string(vt.total_tiles) +
                                     " tiles exceed the static scratch of " + std::to_string(kNoAllocTiles) +
                                     " tiles (use gs_render_fwd with a workspace)");
  float* tl = nullptr;
  if (want_loss && (s = noalloc_scratch(&tl)) != GS_OK) return s;
  return render_fwd_impl(proj, n, bins, cams, n_views, opts, loss, out, vt, tl, as_stream(stream));
}


namespace gs {

static gs_status validate_loss_bwd(const gs_loss* loss, const gs_image* img) {
  if (!loss || (loss->kind != GS_LOSS_L1 && loss->kind != GS_LOSS_EXTERNAL))
    return fail(GS_ERR_INVALID_VALUE, "loss must be GS_LOSS_L1 or GS_LOSS_EXTERNAL");
  if (!img || !img->rgb) return fail(GS_ERR_INVALID_VALUE, "img->rgb (the forward's image) is required");
  if (loss->kind == GS_LOSS_L1 && !loss->target) return fail(GS_ERR_INVALID_VALUE, "L1 loss needs a target");
  if (loss->kind == GS_LOSS_EXTERNAL && !loss->dl_dimage)
    return fail(GS_ERR_INVALID_VALUE, "external loss needs dl_dimage");
  return GS_OK;
}

static gs_status validate_grads(const gs_params* params, const gs_grads* grads) {
  if (!grads || !grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits || !grads->sh_dc ||
      (params->sh_degree > 0 && !grads->sh_rest))
    return fail(GS_ERR_INVALID_VALUE, "a gradient pointer is NULL");
  if (reinterpret_cast<uintptr_t>(grads->quats) % 16 != 0)
    return fail(GS_ERR_INVALID_VALUE, "grads->quats must be 16-byte aligned");
  return GS_OK;
}

static void launch_raster_bwd(const ViewTable& vt, const gs_projected* proj, const gs_bins* bins, const gs_image* img,
                              const gs_options* opts, const gs_loss* loss, float* g2, float* a2, hipStream_t st) {
  const RasterConsts rc = consts_of(opts);
  const dim3 grid((unsigned)vt.total_tiles);
  const ListArgs la = list_args(bins);
  const bool win = (opts->flags & GS_OPT_WINDOW_LISTS) != 0;
#define GS_BWD_W(TILE, ABS, RPL, WIN)                                                                        \
  hipLaunchKernelGGL((k_render_bwd<TILE, ABS, RPL, WIN>), grid, dim3(BwdShape<TILE>::THREADS), 0, st, vt,     \
                     proj->rec, la, rc, img->rgb, (int)loss->kind, loss->target, loss->dl_dimage, g2, a2)
#define GS_BWD_R(TILE, ABS, RPL)      \
  do {                                \
    if (win)                          \
      GS_BWD_W(TILE, ABS, RPL, true); \
    else                              \
      GS_BWD_W(TILE, ABS, RPL, false);\
  } while (0)
#define GS_BWD(TILE, ABS)          \
  do {                             \
    if (opts->lds_batch == 2)      \
      GS_BWD_R(TILE, ABS, 2);      \
    else                           \
      GS_BWD_R(TILE, ABS, 1);      \
  } while (0)
  if (a2) {
    switch (opts->tile_size) {
      case 8: GS_BWD(8, true); break;
      case 16: GS_BWD(16, true); break;
      default: GS_BWD(32, true); break;
    }
  } else {
    switch (opts->tile_size) {
      case 8: GS_BWD(8, false); break;
      case 16: GS_BWD(16, false); break;
      default: GS_BWD(32, false); break;
    }
  }
#undef GS_BWD_W
#undef GS_BWD_R
#undef GS_BWD
}

}  // namespace gs

extern "C" gs_status gs_raster_bwd(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_image* img,
                                   const gs_camera* cams, int32_t n_views, const gs_options* opts,
                                   const gs_loss* loss, float* grad2d, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_raster_common(proj, bins, cams, n_views, opts)) != GS_OK) return s;
  if (n < 1) return fail(GS_ERR_INVALID_VALUE, "n must be >= 1");
  if ((s = validate_loss_bwd(loss, img)) != GS_OK) return s;
  if (!grad2d) return fail(GS_ERR_INVALID_VALUE, "grad2d is NULL");
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  launch_raster_bwd(vt, proj, bins, img, opts, loss, grad2d, nullptr, as_stream(stream));
  return check_launch("raster backward");
}

extern "C" gs_status gs_raster_bwd_abs(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_image* img,
                                       const gs_camera* cams, int32_t n_views, const gs_options* opts,
                                       const gs_loss* loss, float* grad2d, float* abs_grad2d, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_raster_common(proj, bins, cams, n_views, opts)) != GS_OK) return s;
  if (n < 1) return fail(GS_ERR_INVALID_VALUE, "n must be >= 1");
  if ((s = validate_loss_bwd(loss, img)) != GS_OK) return s;
  if (!grad2d || !abs_grad2d) return fail(GS_ERR_INVALID_VALUE, "grad2d and abs_grad2d are required");
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  launch_raster_bwd(vt, proj, bins, img, opts, loss, grad2d, abs_grad2d, as_stream(stream));
  return check_launch("raster backward");
}

extern "C" gs_status gs_project_bwd(const gs_params* params, const gs_projected* proj, const gs_camera* cams,
                                    int32_t n_views, const gs_options* opts, const float* grad2d,
                                    const gs_grads* grads, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_params(params)) != GS_OK) return s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if (!proj || !proj->tiles_touched) return fail(GS_ERR_INVALID_VALUE, "proj->tiles_touched is NULL");
  if (!grad2d) return fail(GS_ERR_INVALID_VALUE, "grad2d is NULL");
  if ((s = validate_grads(params, grads)) != GS_OK) return s;
  return launch_project_bwd(params, cams, n_views, opts, proj->tiles_touched, grad2d, grads, as_stream(stream));
}

extern "C" gs_status gs_render_bwd(const gs_params* params, const gs_projected* proj, const gs_bins* bins,
                                   const gs_image* img, const gs_camera* cams, int32_t n_views, const gs_options* opts,
                                   const gs_loss* loss, const gs_grads* grads, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_params(params)) != GS_OK) return s;
  if ((s = validate_raster_common(proj, bins, cams, n_views, opts)) != GS_OK) return s;
  if ((s = validate_loss_bwd(loss, img)) != GS_OK) return s;
  if ((s = validate_grads(params, grads)) != GS_OK) return s;
  const size_t g2n = (size_t)GS_GRAD2D_FLOATS * (size_t)params->n * (size_t)n_views;
  if (!workspace || workspace_bytes < sizeof(float) * g2n)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(sizeof(float) * g2n) + " bytes");
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  hipStream_t st = as_stream(stream);
  float* g2 = static_cast<float*>(workspace);
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)std::min<size_t>(8192, (g2n + 255) / 256)), dim3(256), 0, st, g2,
                     (uint64_t)g2n);
  launch_raster_bwd(vt, proj, bins, img, opts, loss, g2, nullptr, st);
  if ((s = check_launch("render backward")) != GS_OK) return s;
  return launch_project_bwd(params, cams, n_views, opts, proj->tiles_touched, g2, grads, st);
}

extern "C" gs_status gs_render_stats(const gs_projected* proj, int64_t n, const gs_bins* bins, const gs_camera* cams,
                                     int32_t n_views, const gs_options* opts, int64_t* d_counts, void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_raster_common(proj, bins, cams, n_views, opts)) != GS_OK) return s;
  if (n < 1) return fail(GS_ERR_INVALID_VALUE, "n must be >= 1");
  if (!d_counts) return fail(GS_ERR_INVALID_VALUE, "d_counts is NULL");
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  hipStream_t st = as_stream(stream);
  const RasterConsts rc = consts_of(opts);
  unsigned long long* out = reinterpret_cast<unsigned long long*>(d_counts);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, out, 3);
  const dim3 grid((unsigned)vt.total_tiles);
  const ListArgs la = list_args(bins);
  const bool win = (opts->flags & GS_OPT_WINDOW_LISTS) != 0;
#define GS_STATS(TILE)                                                                                          \
  do {                                                                                                          \
    if (win)                                                                                                    \
      hipLaunchKernelGGL((k_render_stats<TILE, true>), grid, dim3(FwdShape<TILE>::THREADS), 0, st, vt, proj->rec, \
                         la, rc, out);                                                                          \
    else                                                                                                        \
      hipLaunchKernelGGL((k_render_stats<TILE, false>), grid, dim3(FwdShape<TILE>::THREADS), 0, st, vt,          \
                         proj->rec, la, rc, out);                                                               \
  } while (0)
  switch (opts->tile_size) {
    case 8: GS_STATS(8); break;
    case 16: GS_STATS(16); break;
    default: GS_STATS(32); break;
  }
#undef GS_STATS
  return check_launch("render stats");
}
