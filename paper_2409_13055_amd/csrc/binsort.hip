// Tile binning and depth ordering (Sec. II "depth-sorting"; the tile-based
// rasterisation of Sec. III-B).
//
// The required order of the (tile, pair) incidences is that of a stable sort
// on the 64-bit key (global tile << 32 | FP32 bits of the depth) of the
// incidences emitted in (v*N+i) order.  An LSD radix sort processes the key
// from its least significant digit up, and every incidence of one pair shares
// the low 32 key bits; so the depth digits are sorted first over the visible
// (view, Gaussian) pairs only (V*N entries instead of M incidences), the
// incidences are then emitted in that order, and the remaining passes sort
// the tile digits.  The result is identical to the full 64-bit LSD sort while
// moving 12*M bytes per depth digit less.
//
// Every kernel reads its element count from device memory and uses a grid
// sized by the capacity, so the whole call can be captured in a HIP graph
// without a host round trip.
#include <algorithm>
#include <string>

#include "gs_internal.h"

namespace gs {

constexpr int kSortThreads = 256;
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;

struct Chunk {
  uint64_t begin, end;
};
__device__ inline Chunk chunk_of(uint64_t count, int nb, int b) {
  uint64_t per = (count + nb - 1) / nb;
  per = (per + kSortThreads - 1) / kSortThreads * kSortThreads;
  const uint64_t s = std::min<uint64_t>(count, per * (uint64_t)b);
  const uint64_t e = std::min<uint64_t>(count, s + per);
  return {s, e};
}

// Exclusive scan of one value per thread over a 256-thread block.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T* s_wave /*[4]*/, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[w] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T t = s_wave[k];
    off += (k < w) ? t : T(0);
    tot += t;
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

__device__ inline uint32_t depth_key(const float* rec, uint32_t row) {
  return __float_as_uint(rec[(size_t)row * GS_REC_FLOATS + kDepth]);
}

// ---------------------------------------------------------------------------
// Visible-pair compaction: A_key/A_val = (depth bits, v*N+i) of every pair
// with tiles_touched > 0, in (v*N+i) order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_count_visible(const int32_t* __restrict__ tiles, uint64_t count,
                                                                int nb, uint64_t* __restrict__ partial) {
  __shared__ uint64_t s_w[4];
  const Chunk c = chunk_of(count, nb, blockIdx.x);
  uint64_t sum = 0;
  for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += kSortThreads) sum += tiles[i] > 0 ? 1 : 0;
  uint64_t tot;
  block_exclusive_scan<uint64_t>(sum, s_w, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Exclusive scan of the per-block partials in place (single block);
// total -> *total_u64, *out_i64 and (0 when above cap32) *total_u32.
__global__ __launch_bounds__(kSortThreads) void k_scan_partials(uint64_t* __restrict__ partial, int nb,
                                                                uint64_t* __restrict__ total_u64,
                                                                uint32_t* __restrict__ total_u32, uint64_t cap32,
                                                                int64_t* __restrict__ out_i64,
                                                                int32_t* __restrict__ overflow, uint64_t capacity) {
  __shared__ uint64_t s_w[4];
  uint64_t carry = 0;
  for (int base = 0; base < nb; base += kSortThreads) {
    const int i = base + threadIdx.x;
    const uint64_t v = i < nb ? partial[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t>(v, s_w, tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (total_u64) *total_u64 = carry;
    // Past the capacity the outputs are undefined; a zero count makes every
    // later kernel of the call a no-op instead of reading unwritten entries.
    if (total_u32) *total_u32 = carry > cap32 ? 0u : (uint32_t)carry;
    if (out_i64) *out_i64 = (int64_t)carry;
    if (overflow) *overflow = carry > capacity ? 1 : 0;
  }
}

__global__ __launch_bounds__(kSortThreads) void k_compact_visible(const int32_t* __restrict__ tiles,
                                                                  const float* __restrict__ rec, uint64_t count,
                                                                  int nb, const uint64_t* __restrict__ partial,
                                                                  uint32_t* __restrict__ a_key,
                                                                  uint32_t* __restrict__ a_val) {
  __shared__ uint64_t s_w[4];
  const Chunk c = chunk_of(count, nb, blockIdx.x);
  uint64_t run = partial[blockIdx.x];
  for (uint64_t base = c.begin; base < c.end; base += kSortThreads) {
    const uint64_t i = base + threadIdx.x;
    const bool vis = i < c.end && tiles[i] > 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t>(vis ? 1 : 0, s_w, tot);
    if (vis) {
      const uint64_t pos = run + ex;
      a_key[pos] = depth_key(rec, (uint32_t)i);
      a_val[pos] = (uint32_t)i;
    }
    run += tot;
  }
}

// ---------------------------------------------------------------------------
// Stable LSD radix pass (8-bit digit at `shift`) over `*d_count` (key, value)
// pairs: per-block digit histograms, per-digit scan over blocks, then a
// stable block-local ranking (wavefront ballots + per-wave digit counts in
// LDS) and scatter.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ d_count, int shift, int nb,
                                                             uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadixBins];
  h[threadIdx.x] = 0;
  __syncthreads();
  const Chunk c = chunk_of(*d_count, nb, blockIdx.x);
  for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += kSortThreads)
    atomicAdd(&h[(keys[i] >> shift) & (kRadixBins - 1)], 1u);
  __syncthreads();
  hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's per-block counts.
__global__ __launch_bounds__(kSortThreads) void k_radix_scan_digit(uint32_t* __restrict__ hist, int nb,
                                                                   uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t s_w[4];
  uint32_t* h = hist + (size_t)blockIdx.x * nb;
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += kSortThreads) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nb ? h[i] : 0;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(v, s_w, tot);
    if (i < nb) h[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ d_count, int shift, int nb,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t s_base[kRadixBins];
  __shared__ uint32_t s_wcnt[4][kRadixBins];
  __shared__ uint32_t s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  {
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(digit_total[tid], s_w, tot);
    s_base[tid] = ex + hist[(size_t)tid * nb + blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k) s_wcnt[k][tid] = 0;
  }
  __syncthreads();
  const Chunk c = chunk_of(*d_count, nb, blockIdx.x);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (uint64_t base = c.begin; base < c.end; base += kSortThreads) {
    const uint64_t i = base + tid;
    const bool valid = i < c.end;
    const uint32_t k = valid ? kin[i] : 0u;
    const uint32_t val = valid ? vin[i] : 0u;
    const uint32_t d = (k >> shift) & (kRadixBins - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) s_wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = s_base[d] + rank;
      for (int k2 = 0; k2 < w; ++k2) pos += s_wcnt[k2][d];
      kout[pos] = k;
      vout[pos] = val;
    }
    __syncthreads();
    s_base[tid] += s_wcnt[0][tid] + s_wcnt[1][tid] + s_wcnt[2][tid] + s_wcnt[3][tid];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) s_wcnt[k2][tid] = 0;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Incidence counting and emission in depth order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_count_pairs(const int32_t* __restrict__ tiles,
                                                              const uint32_t* __restrict__ sorted_val,
                                                              const uint32_t* __restrict__ d_k, int nb,
                                                              uint64_t* __restrict__ partial) {
  __shared__ uint64_t s_w[4];
  const Chunk c = chunk_of(*d_k, nb, blockIdx.x);
  uint64_t sum = 0;
  for (uint64_t j = c.begin + threadIdx.x; j < c.end; j += kSortThreads) sum += (uint64_t)tiles[sorted_val[j]];
  uint64_t tot;
  block_exclusive_scan<uint64_t>(sum, s_w, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kSortThreads) void k_emit_pairs(
    const int32_t* __restrict__ tiles, const uint32_t* __restrict__ sorted_val, const float* __restrict__ rec,
    const uint32_t* __restrict__ d_k, int nb, const uint64_t* __restrict__ partial, ViewTable vt, uint32_t n,
    uint64_t capacity, uint32_t* __restrict__ p_key, uint32_t* __restrict__ p_val) {
  __shared__ uint64_t s_w[4];
  const Chunk c = chunk_of(*d_k, nb, blockIdx.x);
  uint64_t run = partial[blockIdx.x];
  for (uint64_t base = c.begin; base < c.end; base += kSortThreads) {
    const uint64_t j = base + threadIdx.x;
    uint32_t id = 0;
    uint64_t cnt = 0;
    if (j < c.end) {
      id = sorted_val[j];
      cnt = (uint64_t)tiles[id];
    }
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t>(cnt, s_w, tot);
    uint64_t pos = run + ex;
    if (cnt > 0 && pos + cnt <= capacity) {
      const int v = (int)(id / n);
      const ViewGeom& g = vt.v[v];
      const float4 r0 = reinterpret_cast<const float4*>(rec + (size_t)id * GS_REC_FLOATS)[0];
      const float4 r2 = reinterpret_cast<const float4*>(rec + (size_t)id * GS_REC_FLOATS)[2];
      int x0, y0, x1, y1;
      tile_rect(r0.x, r0.y, __float_as_int(r2.z), vt.tile, g.TX, g.TY, x0, y0, x1, y1);
      for (int ty = y0; ty < y1; ++ty)
        for (int tx = x0; tx < x1; ++tx) {
          p_key[pos] = (uint32_t)(g.tile_off + ty * g.TX + tx);
          p_val[pos] = id;
          ++pos;
        }
    }
    run += tot;
  }
}

// ---------------------------------------------------------------------------
// Tile ranges (+ optional 64-bit keys) from the tile-sorted incidences.
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_ranges(const uint32_t* __restrict__ tkey, const uint32_t* __restrict__ ids,
                         const float* __restrict__ rec, const uint32_t* __restrict__ d_m, uint32_t total_tiles,
                         uint32_t* __restrict__ ranges, uint64_t* __restrict__ keys64) {
  const uint32_t m = *d_m;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
    const uint32_t t = tkey[p];
    if (t >= total_tiles) continue;
    if (p == 0 || tkey[p - 1] != t) ranges[2 * (size_t)t] = p;
    if (p + 1 == m || tkey[p + 1] != t) ranges[2 * (size_t)t + 1] = p + 1;
    if (keys64) keys64[p] = ((uint64_t)t << 32) | depth_key(rec, ids[p]);
  }
}

// ---------------------------------------------------------------------------
// Workspace layout.
// ---------------------------------------------------------------------------
struct SortPlan {
  uint64_t vn;       // n_views * n
  uint64_t cap;      // pair capacity
  int nb_vn;         // blocks over V*N / K entries
  int nb_m;          // blocks over pair entries
  int tile_passes;   // 8-bit tile digits
  size_t off_counters, off_part_a, off_part_b, off_hist, off_dtot;
  size_t off_akey, off_aval, off_bkey, off_bval, off_pkey0, off_pkey1, off_pval;
  size_t bytes;
};

static SortPlan make_plan(int64_t n, int32_t n_views, int64_t total_tiles, int64_t capacity) {
  SortPlan p;
  p.vn = (uint64_t)n * (uint64_t)n_views;
  p.cap = (uint64_t)capacity;
  p.nb_vn = (int)std::min<uint64_t>(1024, std::max<uint64_t>(1, (p.vn + 4095) / 4096));
  p.nb_m = (int)std::min<uint64_t>(2048, std::max<uint64_t>(1, (p.cap + 8191) / 8192));
  int bits = 1;
  while ((int64_t(1) << bits) < total_tiles) ++bits;
  p.tile_passes = (bits + kRadixBits - 1) / kRadixBits;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  p.off_counters = take(64);
  p.off_part_a = take(sizeof(uint64_t) * p.nb_vn);
  p.off_part_b = take(sizeof(uint64_t) * p.nb_vn);
  p.off_hist = take(sizeof(uint32_t) * kRadixBins * std::max(p.nb_vn, p.nb_m));
  p.off_dtot = take(sizeof(uint32_t) * kRadixBins);
  p.off_akey = take(sizeof(uint32_t) * p.vn);
  p.off_aval = take(sizeof(uint32_t) * p.vn);
  p.off_bkey = take(sizeof(uint32_t) * p.vn);
  p.off_bval = take(sizeof(uint32_t) * p.vn);
  p.off_pkey0 = take(sizeof(uint32_t) * std::max<uint64_t>(p.cap, 1));
  p.off_pkey1 = take(sizeof(uint32_t) * std::max<uint64_t>(p.cap, 1));
  p.off_pval = take(sizeof(uint32_t) * std::max<uint64_t>(p.cap, 1));
  p.bytes = o;
  return p;
}

static void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                       const uint32_t* d_count, int shift, int nb, uint32_t* hist, uint32_t* dtot, hipStream_t st) {
  hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortThreads), 0, st, kin, d_count, shift, nb, hist);
  hipLaunchKernelGGL(k_radix_scan_digit, dim3(kRadixBins), dim3(kSortThreads), 0, st, hist, nb, dtot);
  hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortThreads), 0, st, kin, vin, kout, vout, d_count, shift, nb,
                     hist, dtot);
}

}  // namespace gs

extern "C" gs_status gs_bin_sort_workspace_size(int64_t n, const gs_camera* cams, int32_t n_views,
                                                const gs_options* opts, int64_t pair_capacity, size_t* bytes) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if (!bytes) return fail(GS_ERR_INVALID_VALUE, "bytes is NULL");
  if (n < 1 || pair_capacity < 0) return fail(GS_ERR_INVALID_VALUE, "need n >= 1 and pair_capacity >= 0");
  if (pair_capacity >= (int64_t(1) << 32) - 1) return fail(GS_ERR_INVALID_VALUE, "pair_capacity must be < 2^32 - 1");
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  *bytes = make_plan(n, n_views, vt.total_tiles, pair_capacity).bytes;
  return GS_OK;
}

extern "C" gs_status gs_bin_sort(const gs_projected* proj, int64_t n, const gs_camera* cams, int32_t n_views,
                                 const gs_options* opts, const gs_bins* bins, void* workspace, size_t workspace_bytes,
                                 void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if (!proj || !proj->rec || !proj->tiles_touched) return fail(GS_ERR_INVALID_VALUE, "proj is incomplete");
  if (!bins || !bins->ids || !bins->ranges || !bins->d_num_pairs || !bins->d_overflow)
    return fail(GS_ERR_INVALID_VALUE, "bins is incomplete");
  if (n < 1 || (int64_t)n_views * n >= (int64_t(1) << 32) - 1) return fail(GS_ERR_INVALID_VALUE, "bad n");
  if (bins->capacity < 0 || bins->capacity >= (int64_t(1) << 32) - 1)
    return fail(GS_ERR_INVALID_VALUE, "bins->capacity must be in [0, 2^32 - 1)");
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  const SortPlan p = make_plan(n, n_views, vt.total_tiles, bins->capacity);
  if (!workspace || workspace_bytes < p.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(p.bytes) + " bytes");
  hipStream_t st = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  uint64_t* counters = reinterpret_cast<uint64_t*>(ws + p.off_counters);
  uint32_t* d_k = reinterpret_cast<uint32_t*>(counters + 0);        // visible pair count
  uint32_t* d_m = reinterpret_cast<uint32_t*>(counters + 1);        // min(M, capacity)
  uint64_t* part_a = reinterpret_cast<uint64_t*>(ws + p.off_part_a);
  uint64_t* part_b = reinterpret_cast<uint64_t*>(ws + p.off_part_b);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + p.off_hist);
  uint32_t* dtot = reinterpret_cast<uint32_t*>(ws + p.off_dtot);
  uint32_t* akey = reinterpret_cast<uint32_t*>(ws + p.off_akey);
  uint32_t* aval = reinterpret_cast<uint32_t*>(ws + p.off_aval);
  uint32_t* bkey = reinterpret_cast<uint32_t*>(ws + p.off_bkey);
  uint32_t* bval = reinterpret_cast<uint32_t*>(ws + p.off_bval);
  uint32_t* pkey[2] = {reinterpret_cast<uint32_t*>(ws + p.off_pkey0), reinterpret_cast<uint32_t*>(ws + p.off_pkey1)};
  uint32_t* pval_ws = reinterpret_cast<uint32_t*>(ws + p.off_pval);

  // 1. visible (view, Gaussian) pairs, compacted in id order with their depth keys
  hipLaunchKernelGGL(k_count_visible, dim3(p.nb_vn), dim3(kSortThreads), 0, st, proj->tiles_touched, p.vn, p.nb_vn,
                     part_a);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kSortThreads), 0, st, part_a, p.nb_vn, (uint64_t*)nullptr, d_k,
                     (uint64_t)UINT32_MAX, (int64_t*)nullptr, (int32_t*)nullptr, (uint64_t)UINT64_MAX);
  hipLaunchKernelGGL(k_compact_visible, dim3(p.nb_vn), dim3(kSortThreads), 0, st, proj->tiles_touched, proj->rec,
                     p.vn, p.nb_vn, part_a, akey, aval);
  // 2. depth digits (bit 31 of a positive float is 0): four 8-bit passes, ends in (akey, aval)
  radix_pass(akey, aval, bkey, bval, d_k, 0, p.nb_vn, hist, dtot, st);
  radix_pass(bkey, bval, akey, aval, d_k, 8, p.nb_vn, hist, dtot, st);
  radix_pass(akey, aval, bkey, bval, d_k, 16, p.nb_vn, hist, dtot, st);
  radix_pass(bkey, bval, akey, aval, d_k, 24, p.nb_vn, hist, dtot, st);
  // 3. incidence count M, overflow check, emission in depth order
  hipLaunchKernelGGL(k_count_pairs, dim3(p.nb_vn), dim3(kSortThreads), 0, st, proj->tiles_touched, aval, d_k,
                     p.nb_vn, part_b);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kSortThreads), 0, st, part_b, p.nb_vn, (uint64_t*)nullptr, d_m,
                     p.cap, bins->d_num_pairs, bins->d_overflow, p.cap);
  // the last tile pass must land its values in bins->ids
  uint32_t* vbuf[2];
  if (p.tile_passes % 2 == 1) {
    vbuf[0] = pval_ws;
    vbuf[1] = bins->ids;
  } else {
    vbuf[0] = bins->ids;
    vbuf[1] = pval_ws;
  }
  hipLaunchKernelGGL(k_emit_pairs, dim3(p.nb_vn), dim3(kSortThreads), 0, st, proj->tiles_touched, aval, proj->rec,
                     d_k, p.nb_vn, part_b, vt, (uint32_t)n, p.cap, pkey[0], vbuf[0]);
  // 4. tile digits
  for (int k = 0; k < p.tile_passes; ++k)
    radix_pass(pkey[k % 2], vbuf[k % 2], pkey[(k + 1) % 2], vbuf[(k + 1) % 2], d_m, kRadixBits * k, p.nb_m, hist,
               dtot, st);
  // 5. ranges (and the optional 64-bit keys)
  const uint64_t rcount = 2 * (uint64_t)vt.total_tiles;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>(4096, (rcount + 255) / 256)), dim3(256), 0, st,
                     bins->ranges, rcount, 0u);
  const unsigned rg = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(8192, (p.cap + 255) / 256));
  hipLaunchKernelGGL(k_ranges, dim3(rg), dim3(256), 0, st, pkey[p.tile_passes % 2], bins->ids, proj->rec, d_m,
                     (uint32_t)vt.total_tiles, bins->ranges, bins->keys);
  return check_launch("bin/sort");
}
