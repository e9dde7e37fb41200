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

// Exclusive scan of one value per thread over an NT-thread block (NT/64
// wavefronts); `total` receives the block sum.
template <typename T, int NT = kSortThreads>
__device__ inline T block_exclusive_scan(T v, T* s_wave /*[NT/64]*/, T& total) {
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
  for (int k = 0; k < NT / 64; ++k) {
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
  // eight loads in flight per thread, then their LDS increments
  constexpr int U = 8;
  uint64_t i = c.begin + threadIdx.x;
  for (; i + (U - 1) * kSortThreads < c.end; i += U * kSortThreads) {
    uint32_t k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) k[u] = keys[i + (uint64_t)u * kSortThreads];
#pragma unroll
    for (int u = 0; u < U; ++u) atomicAdd(&h[(k[u] >> shift) & (kRadixBins - 1)], 1u);
  }
  for (; i < c.end; i += kSortThreads) atomicAdd(&h[(keys[i] >> shift) & (kRadixBins - 1)], 1u);
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

// Downsweep: a block ranks a tile of kTileKeys keys at a time.  Wave w owns
// the tile's keys [w*512, (w+1)*512) as 8 groups of 64; ballots over the 8
// digit bits give each key its rank among equal digits of its group, and a
// per-wave digit counter in LDS carries the rank across groups (a wave's LDS
// operations execute in program order, so no barrier is needed).  The tile is
// then reordered by digit in LDS and written out digit run by digit run, so
// global stores are coalesced.  Order inside a digit follows the input index,
// which keeps every pass stable.
constexpr int kItems = 8;
constexpr int kTileKeys = kSortThreads * kItems;

// Emission of the (tile, pair) incidences in depth order (pair order, tiles
// row-major inside each pair's rect), generated on the fly from per-pair
// offsets: see k_entry_offsets.  The first tile-digit pass reads its input
// from here instead of from an emitted array.
constexpr int kChunk = kItems;  // output slots per chunk_start entry: one thread's run
struct EmitSrc {
  const uint32_t* d_k;          // number of depth-ordered visible pairs
  const uint64_t* ent_off;      // exclusive incidence offset per pair
  const uint4* ent_rec;         // per pair: (global tile of the rect's top-left, TX | width << 16, id, tiles)
  const uint32_t* chunk_start;  // pair holding slot c * kChunk
};

// Incidences q0 .. q0 + R - 1 into (kk, vv), q0 a multiple of kChunk; slots
// at or past `end` (<= M) are left unset.  The owner of slot q0 comes from
// the chunk table, then the run walks the rects, one pair record ahead.
template <int R>
__device__ __forceinline__ void emit_run(const EmitSrc& es, uint32_t K, uint64_t q0, uint64_t end, uint32_t* kk,
                                         uint32_t* vv) {
  if (q0 >= end) return;
  uint32_t j = es.chunk_start[q0 / kChunk];
  const uint64_t start = es.ent_off[j];
  uint4 r = es.ent_rec[j];
  uint4 rn = (j + 1 < K) ? es.ent_rec[j + 1] : r;
  uint64_t next = start + r.w;
  uint32_t w = r.y >> 16;
  const uint32_t k0 = (uint32_t)(q0 - start);
  uint32_t ty = k0 / w, tx = k0 - ty * w;
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const uint64_t q = q0 + e;
    if (q < end) {
      while (q >= next) {  // next pair (every listed pair has at least one tile)
        ++j;
        r = rn;
        next += r.w;
        rn = (j + 1 < K) ? es.ent_rec[j + 1] : r;
        w = r.y >> 16;
        tx = ty = 0;
      }
    }
    kk[e] = r.x + ty * (r.y & 0xffffu) + tx;
    vv[e] = r.z;
    if (++tx == w) {
      tx = 0;
      ++ty;
    }
  }
}

// Digit histogram of the emitted incidences (the input of the first tile pass).
__global__ __launch_bounds__(kSortThreads) void k_emit_hist(EmitSrc es, const uint32_t* __restrict__ d_m, int shift,
                                                            int nb, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadixBins];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t K = *es.d_k;
  const uint64_t M = *d_m;
  const Chunk c = chunk_of(M, nb, blockIdx.x);
  for (uint64_t tb = c.begin; tb < c.end; tb += kTileKeys) {
    uint32_t kk[kItems], vv[kItems];
    const uint64_t q0 = tb + (uint64_t)threadIdx.x * kItems;
    emit_run<kItems>(es, K, q0, c.end, kk, vv);
#pragma unroll
    for (int e = 0; e < kItems; ++e)
      if (q0 + e < c.end) atomicAdd(&h[(kk[e] >> shift) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// EMIT: the input tile is generated by emit_run (natural order, staged in LDS)
// instead of being read from (kin, vin).
template <bool EMIT>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, EmitSrc es, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ d_count, int shift, int nb,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ digit_total, uint64_t* __restrict__ keys64,
    const float* __restrict__ rec) {
  __shared__ uint32_t s_keys[kTileKeys];
  __shared__ uint32_t s_vals[kTileKeys];
  __shared__ uint32_t s_wc[4][kRadixBins];
  __shared__ uint32_t s_start[kRadixBins];
  __shared__ uint32_t s_glob[kRadixBins];
  __shared__ uint32_t s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  {
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(digit_total[tid], s_w, tot);
    s_glob[tid] = ex + hist[(size_t)tid * nb + blockIdx.x];
  }
  const uint64_t count = *d_count;
  const uint32_t K = EMIT ? *es.d_k : 0u;
  const Chunk c = chunk_of(count, nb, blockIdx.x);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // item k of lane `lane` in wave w sits at tile offset w*(kItems*64) + k*64 + lane
  const uint32_t o0 = (uint32_t)w * (kItems * 64) + (uint32_t)lane;
  for (uint64_t tb = c.begin; tb < c.end; tb += kTileKeys) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_wc[k][tid] = 0;
    if (EMIT) {
      uint32_t kk[kItems], vv[kItems];
      emit_run<kItems>(es, K, tb + (uint64_t)tid * kItems, c.end, kk, vv);
      uint4* sk = reinterpret_cast<uint4*>(s_keys) + tid * (kItems / 4);
      uint4* sv = reinterpret_cast<uint4*>(s_vals) + tid * (kItems / 4);
#pragma unroll
      for (int q = 0; q < kItems / 4; ++q) {
        sk[q] = make_uint4(kk[4 * q], kk[4 * q + 1], kk[4 * q + 2], kk[4 * q + 3]);
        sv[q] = make_uint4(vv[4 * q], vv[4 * q + 1], vv[4 * q + 2], vv[4 * q + 3]);
      }
    }
    __syncthreads();
    uint32_t key[kItems], val[kItems], rk[kItems];
    const uint64_t lim = c.end - tb;  // keys left from this tile's start
    if (!EMIT) {
      // all of the tile's loads first, unconditionally (indices clamped into the tile), so they are
      // in flight together rather than one dependent round trip per item
      const uint32_t* kt = kin + tb;
      const uint32_t* vt = vin + tb;
      const uint32_t last = (uint32_t)min<uint64_t>(lim, (uint64_t)kTileKeys) - 1;
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const uint32_t o = min(o0 + (uint32_t)k * 64, last);
        key[k] = kt[o];
        val[k] = vt[o];
      }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const uint32_t o = o0 + (uint32_t)k * 64;
      const bool valid = o < lim;
      if (EMIT) {
        key[k] = valid ? s_keys[o] : 0u;
        val[k] = valid ? s_vals[o] : 0u;
      } else if (!valid) {
        key[k] = 0u;
        val[k] = 0u;
      }
      const uint32_t d = (key[k] >> shift) & (kRadixBins - 1);
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kRadixBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      const uint32_t r = (uint32_t)__popcll(peers & lt);
      const uint32_t before = s_wc[w][d];
      if (valid && r == 0) s_wc[w][d] = before + (uint32_t)__popcll(peers);
      rk[k] = valid ? before + r : 0xffffffffu;
    }
    __syncthreads();
    // thread d: wave prefixes of digit d (in place) and the tile's digit starts
    uint32_t tot_d;
    {
      const uint32_t c0 = s_wc[0][tid], c1 = s_wc[1][tid], c2 = s_wc[2][tid], c3 = s_wc[3][tid];
      tot_d = c0 + c1 + c2 + c3;
      s_wc[0][tid] = 0;
      s_wc[1][tid] = c0;
      s_wc[2][tid] = c0 + c1;
      s_wc[3][tid] = c0 + c1 + c2;
      uint32_t all;
      s_start[tid] = block_exclusive_scan<uint32_t>(tot_d, s_w, all);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (rk[k] != 0xffffffffu) {
        const uint32_t d = (key[k] >> shift) & (kRadixBins - 1);
        const uint32_t lp = s_start[d] + s_wc[w][d] + rk[k];
        s_keys[lp] = key[k];
        s_vals[lp] = val[k];
      }
    }
    __syncthreads();
    const uint32_t n_in = (uint32_t)min<uint64_t>(kTileKeys, c.end - tb);
    for (int k = 0; k < kItems; ++k) {
      const uint32_t i = (uint32_t)tid + (uint32_t)k * kSortThreads;
      if (i < n_in) {
        const uint32_t kk = s_keys[i];
        const uint32_t d = (kk >> shift) & (kRadixBins - 1);
        const uint32_t g = s_glob[d] + (i - s_start[d]);
        const uint32_t vv = s_vals[i];
        if (kout) kout[g] = kk;
        vout[g] = vv;
        if (keys64) keys64[g] = ((uint64_t)kk << 32) | depth_key(rec, vv);
      }
    }
    __syncthreads();
    s_glob[tid] += tot_d;
  }
}

// ---------------------------------------------------------------------------
// Incidence counting and emission in depth order.
// ---------------------------------------------------------------------------
// Incidence counts per step of kStep consecutive depth-ordered pairs.
constexpr int kStep = kSortThreads;
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kSortThreads) void k_step_pair_counts(const int32_t* __restrict__ tiles,
                                                                   const uint32_t* __restrict__ sorted_val,
                                                                   const uint32_t* __restrict__ d_k,
                                                                   uint64_t* __restrict__ step_sums) {
  __shared__ uint64_t s_w[kSortThreads / 64];
  const uint32_t K = *d_k, nsteps = (K + kStep - 1) / kStep;
  for (uint32_t st = blockIdx.x; st < nsteps; st += gridDim.x) {
    const uint32_t j = st * kStep + threadIdx.x;
    const uint64_t cnt = j < K ? (uint64_t)tiles[sorted_val[j]] : 0;
    uint64_t tot;
    block_exclusive_scan<uint64_t>(cnt, s_w, tot);
    if (threadIdx.x == 0) step_sums[st] = tot;
  }
}

// Exclusive scan of the step sums in place (one block); M -> d_num_pairs,
// overflow flag, and the clamped count for the tile passes (0 on overflow).
__global__ __launch_bounds__(kScanThreads) void k_scan_steps(uint64_t* __restrict__ step_sums,
                                                             const uint32_t* __restrict__ d_k,
                                                             uint32_t* __restrict__ d_m, int64_t* __restrict__ d_pairs,
                                                             int32_t* __restrict__ d_overflow, uint64_t capacity) {
  __shared__ uint64_t s_w[kScanThreads / 64];
  const uint32_t nsteps = (*d_k + kStep - 1) / kStep;
  uint64_t carry = 0;
  for (uint32_t base = 0; base < nsteps; base += kScanThreads) {
    const uint32_t i = base + threadIdx.x;
    const uint64_t v = i < nsteps ? step_sums[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t, kScanThreads>(v, s_w, tot);
    if (i < nsteps) step_sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    *d_pairs = (int64_t)carry;
    *d_overflow = carry > capacity ? 1 : 0;
    // past the capacity the outputs are undefined; a zero count makes the
    // remaining kernels of the call no-ops
    *d_m = carry > capacity ? 0u : (uint32_t)carry;
  }
}

// Emission offsets: k_entry_offsets gives every depth-ordered pair its
// exclusive incidence offset and a compact description of its tile rect, and
// records which pair holds the first slot of every kChunk-slot run of the
// output; emit_run then looks up the owner of a run's first slot and walks
// the rects row-major from there, so the work per output slot is fixed
// however skewed the per-pair tile counts are, and the order is that of a
// sequential emission (pair order, tiles row-major within a pair).
__global__ __launch_bounds__(kSortThreads) void k_entry_offsets(
    const int32_t* __restrict__ tiles, const uint32_t* __restrict__ sorted_val, const float* __restrict__ rec,
    const uint32_t* __restrict__ d_k, const uint64_t* __restrict__ step_off, ViewTable vt, uint32_t n,
    uint64_t capacity, uint64_t* __restrict__ ent_off, uint4* __restrict__ ent_rec,
    uint32_t* __restrict__ chunk_start) {
  __shared__ uint64_t s_w[kSortThreads / 64];
  const uint32_t K = *d_k, nsteps = (K + kStep - 1) / kStep;
  for (uint32_t st = blockIdx.x; st < nsteps; st += gridDim.x) {
    const uint32_t j = st * kStep + threadIdx.x;
    uint64_t cnt = 0;
    uint32_t id = 0;
    if (j < K) {
      id = sorted_val[j];
      cnt = (uint64_t)tiles[id];
    }
    uint64_t tot;
    const uint64_t off = step_off[st] + block_exclusive_scan<uint64_t>(cnt, s_w, tot);
    if (j < K) {
      const ViewGeom& g = vt.v[id / n];
      const float4 r0 = reinterpret_cast<const float4*>(rec + (size_t)id * GS_REC_FLOATS)[0];
      const float4 r2 = reinterpret_cast<const float4*>(rec + (size_t)id * GS_REC_FLOATS)[2];
      int x0, y0, x1, y1;
      tile_rect(r0.x, r0.y, ext_x(__float_as_int(r2.z)), ext_y(__float_as_int(r2.z)), vt.tile, g.TX, g.TY, x0, y0,
              x1, y1);
      ent_off[j] = off;
      ent_rec[j] = make_uint4((uint32_t)(g.tile_off + y0 * g.TX + x0), (uint32_t)g.TX | ((uint32_t)(x1 - x0) << 16),
                              id, (uint32_t)cnt);
      // chunk boundaries inside [off, off + cnt): this pair holds their first slot
      if (off + cnt <= capacity)
        for (uint64_t c = (off + kChunk - 1) / kChunk; c * kChunk < off + cnt; ++c) chunk_start[c] = j;
    }
  }
}

// Tile coverage counts: every visible pair adds +1/-1 at the four corners of
// its tile rect in its view's (TX+1) x (TY+1) difference grid, whose 2D
// prefix sum (k_tile_counts) is the number of rects covering each tile.  A
// corner in column TX or row TY only reaches cells outside every tile's
// prefix, so it is dropped.  Block (b, v) takes kCoverPairs consecutive pairs
// of view v and, when `priv` (every view's grid fits the dynamic LDS the
// launch gives), accumulates in a private LDS copy of the grid, then adds its
// non-zero cells to the global grid: device-wide atomics are resolved beyond
// the per-XCD L2, so they are kept few and spread.  Otherwise the corners go
// to the global grid directly.
constexpr int kCoverPairs = 8192;
constexpr int kCoverLdsCells = 16384;

__global__ __launch_bounds__(kSortThreads) void k_cover_counts(const int32_t* __restrict__ tiles,
                                                               const float* __restrict__ rec, ViewTable vt,
                                                               uint32_t n, int priv, int32_t* __restrict__ cover) {
  extern __shared__ int32_t s_grid[];
  const int v = blockIdx.y;
  const ViewGeom& g = vt.v[v];
  const int gw = g.TX + 1, cells = gw * (g.TY + 1);
  int32_t* cg = cover + g.grid_off;
  int32_t* grid = priv ? s_grid : cg;
  if (priv) {
    for (int c = threadIdx.x; c < cells; c += kSortThreads) s_grid[c] = 0;
    __syncthreads();
  }
  const uint64_t i0 = (uint64_t)blockIdx.x * kCoverPairs;
  const uint64_t i1 = min<uint64_t>((uint64_t)n, i0 + kCoverPairs);
  for (uint64_t i = i0 + threadIdx.x; i < i1; i += kSortThreads) {
    const size_t id = (size_t)v * n + i;
    if (tiles[id] <= 0) continue;
    const float4 r0 = reinterpret_cast<const float4*>(rec + id * GS_REC_FLOATS)[0];
    const float4 r2 = reinterpret_cast<const float4*>(rec + id * GS_REC_FLOATS)[2];
    int x0, y0, x1, y1;
    tile_rect(r0.x, r0.y, ext_x(__float_as_int(r2.z)), ext_y(__float_as_int(r2.z)), vt.tile, g.TX, g.TY, x0, y0,
              x1, y1);
    atomicAdd(grid + y0 * gw + x0, 1);
    if (x1 < g.TX) atomicAdd(grid + y0 * gw + x1, -1);
    if (y1 < g.TY) atomicAdd(grid + y1 * gw + x0, -1);
    if (x1 < g.TX && y1 < g.TY) atomicAdd(grid + y1 * gw + x1, 1);
  }
  if (priv) {
    __syncthreads();
    for (int c = threadIdx.x; c < cells; c += kSortThreads) {
      const int32_t d = s_grid[c];
      if (d != 0) atomicAdd(cg + c, d);
    }
  }
}

// Per-view 2D inclusive prefix of the coverage difference grid: the number of
// pair rects covering each tile, i.e. the tile's incidence count.  One block
// per view (rows, then columns).
__global__ __launch_bounds__(kSortThreads) void k_tile_counts(ViewTable vt, int32_t* __restrict__ cover) {
  const ViewGeom& g = vt.v[blockIdx.x];
  int32_t* cg = cover + g.grid_off;
  const int gw = g.TX + 1, gh = g.TY + 1;
  for (int y = threadIdx.x; y < gh; y += kSortThreads) {
    int32_t acc = 0;
    for (int x = 0; x < gw; ++x) {
      acc += cg[y * gw + x];
      cg[y * gw + x] = acc;
    }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < gw; x += kSortThreads) {
    int32_t acc = 0;
    for (int y = 0; y < gh; ++y) {
      acc += cg[y * gw + x];
      cg[y * gw + x] = acc;
    }
  }
}

// ranges[t] = [start, start + count) with start the exclusive prefix of the
// tile counts in global tile order, (0,0) for an empty tile.  One block.
__global__ __launch_bounds__(kScanThreads) void k_ranges_from_counts(ViewTable vt, const int32_t* __restrict__ cover,
                                                                      const uint32_t* __restrict__ d_m,
                                                                      uint32_t* __restrict__ ranges) {
  __shared__ uint64_t s_w[kScanThreads / 64];
  if (*d_m == 0) {  // no pairs, or the pair capacity overflowed
    for (int t = threadIdx.x; t < vt.total_tiles; t += kScanThreads) ranges[2 * t] = ranges[2 * t + 1] = 0;
    return;
  }
  uint64_t carry = 0;
  int v = 0;
  for (int base = 0; base < vt.total_tiles; base += kScanThreads) {
    const int t = base + threadIdx.x;
    uint32_t cnt = 0;
    if (t < vt.total_tiles) {
      while (v + 1 < vt.n_views && vt.v[v + 1].tile_off <= t) ++v;
      const ViewGeom& g = vt.v[v];
      const int lt = t - g.tile_off, ty = lt / g.TX, tx = lt - ty * g.TX;
      cnt = (uint32_t)cover[g.grid_off + ty * (g.TX + 1) + tx];
    }
    uint64_t tot;
    const uint64_t ex = carry + block_exclusive_scan<uint64_t, kScanThreads>(cnt, s_w, tot);
    if (t < vt.total_tiles) {
      ranges[2 * t] = cnt ? (uint32_t)ex : 0u;
      ranges[2 * t + 1] = cnt ? (uint32_t)(ex + cnt) : 0u;
    }
    carry += tot;
  }
}

// ---------------------------------------------------------------------------
// Tile ranges (+ optional 64-bit keys) from the tile-sorted incidences.
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---------------------------------------------------------------------------
// Workspace layout.
// ---------------------------------------------------------------------------
struct SortPlan {
  uint64_t vn;       // n_views * n
  uint64_t cap;      // pair capacity
  int nb_vn;         // blocks over V*N / K entries
  int nb_m;          // blocks over pair entries
  int n_steps;       // kStep-entry steps over V*N
  int grid_steps;    // blocks striding over the steps
  int tile_passes;   // 8-bit tile digits
  size_t off_counters, off_part_a, off_steps, off_hist, off_dtot, off_eoff, off_erec, off_chunks, off_cover;
  size_t off_akey, off_aval, off_bkey, off_bval, off_pkey0, off_pkey1, off_pval;
  size_t bytes;
};

static SortPlan make_plan(int64_t n, int32_t n_views, int64_t total_tiles, int64_t total_grid, int64_t capacity) {
  SortPlan p;
  p.vn = (uint64_t)n * (uint64_t)n_views;
  p.cap = (uint64_t)capacity;
  p.nb_vn = (int)std::min<uint64_t>(4096, std::max<uint64_t>(1, (p.vn + 1023) / 1024));
  p.nb_m = (int)std::min<uint64_t>(4096, std::max<uint64_t>(1, (p.cap + 2047) / 2048));
  p.n_steps = (int)((p.vn + kStep - 1) / kStep);
  p.grid_steps = std::min(p.n_steps, 8192);
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
  p.off_steps = take(sizeof(uint64_t) * p.n_steps);
  p.off_eoff = take(sizeof(uint64_t) * p.vn);
  p.off_erec = take(sizeof(uint4) * p.vn);
  p.off_chunks = take(sizeof(uint32_t) * (p.cap / kChunk + 2));
  p.off_cover = take(sizeof(int32_t) * (size_t)total_grid);
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
                       const uint32_t* d_count, int shift, int nb, uint32_t* hist, uint32_t* dtot, hipStream_t st,
                       uint64_t* keys64 = nullptr, const float* rec = nullptr) {
  hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortThreads), 0, st, kin, d_count, shift, nb, hist);
  hipLaunchKernelGGL(k_radix_scan_digit, dim3(kRadixBins), dim3(kSortThreads), 0, st, hist, nb, dtot);
  hipLaunchKernelGGL(k_radix_scatter<false>, dim3(nb), dim3(kSortThreads), 0, st, kin, vin, EmitSrc{}, kout, vout,
                     d_count, shift, nb, hist, dtot, keys64, rec);
}

// The first tile-digit pass over the incidences generated by emission.
static void radix_pass_emit(const EmitSrc& es, uint32_t* kout, uint32_t* vout, const uint32_t* d_m, int shift,
                            int nb, uint32_t* hist, uint32_t* dtot, hipStream_t st, uint64_t* keys64,
                            const float* rec) {
  hipLaunchKernelGGL(k_emit_hist, dim3(nb), dim3(kSortThreads), 0, st, es, d_m, shift, nb, hist);
  hipLaunchKernelGGL(k_radix_scan_digit, dim3(kRadixBins), dim3(kSortThreads), 0, st, hist, nb, dtot);
  hipLaunchKernelGGL(k_radix_scatter<true>, dim3(nb), dim3(kSortThreads), 0, st, (const uint32_t*)nullptr,
                     (const uint32_t*)nullptr, es, kout, vout, d_m, shift, nb, hist, dtot, keys64, rec);
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
  *bytes = make_plan(n, n_views, vt.total_tiles, vt.total_grid, pair_capacity).bytes;
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
  const SortPlan p = make_plan(n, n_views, vt.total_tiles, vt.total_grid, bins->capacity);
  if (!workspace || workspace_bytes < p.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(p.bytes) + " bytes");
  hipStream_t st = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  uint64_t* counters = reinterpret_cast<uint64_t*>(ws + p.off_counters);
  uint32_t* d_k = reinterpret_cast<uint32_t*>(counters + 0);        // visible pair count
  uint32_t* d_m = reinterpret_cast<uint32_t*>(counters + 1);        // min(M, capacity)
  uint64_t* part_a = reinterpret_cast<uint64_t*>(ws + p.off_part_a);
  uint64_t* step_off = reinterpret_cast<uint64_t*>(ws + p.off_steps);
  uint64_t* ent_off = reinterpret_cast<uint64_t*>(ws + p.off_eoff);
  uint4* ent_rec = reinterpret_cast<uint4*>(ws + p.off_erec);
  uint32_t* chunk_start = reinterpret_cast<uint32_t*>(ws + p.off_chunks);
  int32_t* cover = reinterpret_cast<int32_t*>(ws + p.off_cover);
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
  hipLaunchKernelGGL(k_step_pair_counts, dim3(p.grid_steps), dim3(kSortThreads), 0, st, proj->tiles_touched, aval,
                     d_k, step_off);
  hipLaunchKernelGGL(k_scan_steps, dim3(1), dim3(kScanThreads), 0, st, step_off, d_k, d_m, bins->d_num_pairs,
                     bins->d_overflow, p.cap);
  // the last tile pass must land its values in bins->ids
  uint32_t* vbuf[2];
  if (p.tile_passes % 2 == 1) {
    vbuf[0] = pval_ws;
    vbuf[1] = bins->ids;
  } else {
    vbuf[0] = bins->ids;
    vbuf[1] = pval_ws;
  }
  const uint64_t gcount = (uint64_t)vt.total_grid;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>(4096, (gcount + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<uint32_t*>(cover), gcount, 0u);
  int max_cells = 0;
  for (int v = 0; v < n_views; ++v) max_cells = std::max(max_cells, (vt.v[v].TX + 1) * (vt.v[v].TY + 1));
  const int priv = max_cells <= kCoverLdsCells ? 1 : 0;
  hipLaunchKernelGGL(k_cover_counts, dim3((unsigned)((n + kCoverPairs - 1) / kCoverPairs), (unsigned)n_views),
                     dim3(kSortThreads), priv ? sizeof(int32_t) * (size_t)max_cells : 0, st, proj->tiles_touched,
                     proj->rec, vt, (uint32_t)n, priv, cover);
  hipLaunchKernelGGL(k_entry_offsets, dim3(p.grid_steps), dim3(kSortThreads), 0, st, proj->tiles_touched, aval,
                     proj->rec, d_k, step_off, vt, (uint32_t)n, p.cap, ent_off, ent_rec, chunk_start);
  // 4. tile ranges from the per-tile incidence counts (rect coverage)
  hipLaunchKernelGGL(k_tile_counts, dim3(n_views), dim3(kSortThreads), 0, st, vt, cover);
  hipLaunchKernelGGL(k_ranges_from_counts, dim3(1), dim3(kScanThreads), 0, st, vt, cover, d_m, bins->ranges);
  // 5. tile digits, the first pass fed by emission; the last pass writes only the ids (and the optional
  //    64-bit keys)
  const EmitSrc es{d_k, ent_off, ent_rec, chunk_start};
  for (int k = 0; k < p.tile_passes; ++k) {
    const bool last = k + 1 == p.tile_passes;
    uint32_t* kout = last ? nullptr : pkey[(k + 1) % 2];
    uint64_t* k64 = last ? bins->keys : nullptr;
    if (k == 0)
      radix_pass_emit(es, kout, vbuf[(k + 1) % 2], d_m, 0, p.nb_m, hist, dtot, st, k64, proj->rec);
    else
      radix_pass(pkey[k % 2], vbuf[k % 2], kout, vbuf[(k + 1) % 2], d_m, kRadixBits * k, p.nb_m, hist, dtot, st, k64,
                 proj->rec);
  }
  return check_launch("bin/sort");
}
