// Tile binning and depth ordering (Sec. II, second stage of the rasteriser;
// the tile-based rasterisation of Sec. III-B).
//
// The required order of the (tile, pair) incidences is that of a stable sort
// on the 64-bit key (global tile << 32 | FP32 bits of the depth) of the
// incidences emitted in (v*N+i) order: per tile, the pairs covering it in
// depth order, ties in id order.  The depth digits are sorted once over the
// visible (view, Gaussian) pairs (a stable LSD radix sort, V*N entries instead
// of M incidences).  The tiles are then handled by binning windows of 8x8
// tiles: the depth-ordered pairs are listed in every window their rect meets
// (a short stable sort on the window index), and one wavefront per chunk of a
// window's list writes the ids straight into their final slots, one lane per
// tile, from per-chunk tile counts and the tile ranges.  No pass ever moves
// the M incidences.
//
// Every kernel reads its element count from device memory and uses a grid
// sized by the capacity, so the whole call can be captured in a HIP graph
// without a host round trip.
#include <algorithm>
#include <string>
#include <type_traits>

#include "gs_internal.h"

namespace gs {

constexpr int kSortThreads = 256;
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kScanThreads = 1024;

// A radix block ranks kRadixTile keys at a time; each block's share of the
// keys is a whole number of such tiles (a partial tile costs a full one).
constexpr int kRadixTile = kSortThreads * 8;

struct Chunk {
  uint64_t begin, end;
};
__device__ inline Chunk chunk_of(uint64_t count, int nb, int b) {
  uint64_t per = (count + nb - 1) / nb;
  per = (per + kRadixTile - 1) / kRadixTile * kRadixTile;
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

// Entry record of a visible pair: x = x0 | x1 << 16 and y = y0 | y1 << 16
// (its tile rect [x0,x1) x [y0,y1) in its view's grid), z = v*N+i,
// w = FP32 bits of its depth.
__device__ inline uint32_t rect_windows(uint4 e) {
  const uint32_t x0 = e.x & 0xffffu, x1 = e.x >> 16, y0 = e.y & 0xffffu, y1 = e.y >> 16;
  if (x1 <= x0 || y1 <= y0) return 0;
  return (((x1 - 1) >> kWinShift) - (x0 >> kWinShift) + 1) * (((y1 - 1) >> kWinShift) - (y0 >> kWinShift) + 1);
}
__device__ inline uint32_t rect_tiles(uint4 e) {
  const uint32_t x0 = e.x & 0xffffu, x1 = e.x >> 16, y0 = e.y & 0xffffu, y1 = e.y >> 16;
  return (x1 > x0 && y1 > y0) ? (x1 - x0) * (y1 - y0) : 0u;
}

// Per-view fields indexed by a per-lane view inside a kernel, copied to LDS
// once per block: a lane-indexed read of the kernel-argument table is a
// vector memory load, whose wait would also wait for every store issued
// before it.
struct ViewLds {
  int32_t a[GS_MAX_VIEWS], b[GS_MAX_VIEWS];
};

// Sixteen bytes held in registers or LDS (a plain struct: register arrays of
// HIP's vector types can end up in scratch memory).
struct alignas(16) Words4 {
  uint32_t x, y, z, w;
};

// ---------------------------------------------------------------------------
// Visible-pair compaction from the projection's segments (64 Gaussians of one
// view each, in (v*N+i) order): pair c of the concatenation gets a_key[c] =
// depth bits and entc[c] = its entry record (the first depth pass takes c itself
// as the value carried with key c).
// ---------------------------------------------------------------------------
constexpr int kCopyBatch = 8;  // segments whose entries a wavefront loads before storing any

// Per block of kSortThreads segments: the total of their counts.
__global__ __launch_bounds__(kSortThreads) void k_segment_totals(const uint32_t* __restrict__ seg_count,
                                                                 uint32_t n_seg, uint64_t* __restrict__ partial) {
  __shared__ uint64_t s_w[kSortThreads / 64];
  const uint32_t sg = blockIdx.x * kSortThreads + threadIdx.x;
  uint64_t tot;
  block_exclusive_scan<uint64_t>(sg < n_seg ? seg_count[sg] : 0u, s_w, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Exclusive scan of the per-block partials in place (single block);
// total -> *total_u32 (0 when above cap32).  Each thread takes kScanItems
// consecutive values per round, so a round covers kScanItems blocks' worth of
// values with one block-wide scan.
constexpr int kScanItems = 8;
__global__ __launch_bounds__(kSortThreads) void k_scan_partials(uint64_t* __restrict__ partial, int nb,
                                                                uint32_t* __restrict__ total_u32, uint64_t cap32) {
  __shared__ uint64_t s_w[4];
  uint64_t carry = 0;
  for (int base = 0; base < nb; base += kSortThreads * kScanItems) {
    const int i0 = base + (int)threadIdx.x * kScanItems;
    uint64_t v[kScanItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = i0 + k < nb ? partial[i0 + k] : 0;
      sum += v[k];
    }
    uint64_t tot;
    uint64_t run = carry + block_exclusive_scan<uint64_t>(sum, s_w, tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (i0 + k < nb) partial[i0 + k] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) *total_u32 = carry > cap32 ? 0u : (uint32_t)carry;
}

// Block b copies segments [b kSortThreads, (b + 1) kSortThreads), whose
// entries are the output positions [partial[b], partial[b] + total): wavefront
// w takes the block's segments [64 w, 64 w + 64), kCopyBatch at a time, one
// lane per entry of a segment, so each segment is one contiguous load and one
// contiguous store; the kCopyBatch segments' loads are in flight before any
// of their stores.
__global__ __launch_bounds__(kSortThreads) void k_compact_segments(const uint4* __restrict__ seg_ent,
                                                                   const uint32_t* __restrict__ seg_count,
                                                                   uint32_t n_seg,
                                                                   const uint64_t* __restrict__ partial,
                                                                   uint32_t* __restrict__ a_key,
                                                                   uint4* __restrict__ entc) {
  __shared__ uint32_t s_w[kSortThreads / 64];
  __shared__ uint32_t s_loc[kSortThreads];
  __shared__ uint32_t s_cnt[kSortThreads];
  const uint32_t sg0 = blockIdx.x * kSortThreads;
  const uint32_t c = sg0 + threadIdx.x < n_seg ? seg_count[sg0 + threadIdx.x] : 0u;  // 0 past the last segment
  uint32_t tot;
  s_loc[threadIdx.x] = block_exclusive_scan<uint32_t>(c, s_w, tot);  // at most 256 * 64
  s_cnt[threadIdx.x] = c;
  const uint32_t base = (uint32_t)partial[blockIdx.x];  // < n_views * n < 2^32
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63;
  const int q_begin = (int)(threadIdx.x >> 6) * 64;
  for (int q0 = q_begin; q0 < q_begin + 64; q0 += kCopyBatch) {
    Words4 e[kCopyBatch];
#pragma unroll
    for (int k = 0; k < kCopyBatch; ++k) {
      if (lane < s_cnt[q0 + k]) {
        const uint4 g = seg_ent[(size_t)(sg0 + q0 + k) * 64 + lane];
        e[k] = Words4{g.x, g.y, g.z, g.w};
      }
    }
#pragma unroll
    for (int k = 0; k < kCopyBatch; ++k) {
      if (lane < s_cnt[q0 + k]) {
        const uint32_t pos = base + s_loc[q0 + k] + lane;
        a_key[pos] = e[k].w;
        entc[pos] = make_uint4(e[k].x, e[k].y, e[k].z, e[k].w);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Stable LSD radix pass (8-bit digit at `shift`) over `*d_count` (key, value)
// pairs: per-block digit histograms, per-digit scan over blocks, then a
// stable block-local ranking (wavefront ballots + per-wave digit counts in
// LDS) and scatter.
// ---------------------------------------------------------------------------
// One count of digit d into the block histogram h.  PEERS: the lanes of the
// wavefront holding the same digit (found by ballots over its bits) are added
// by the first of them with one atomic, for a digit with few distinct values
// across the keys (the top digit of depths spanning a narrow range), where
// many lanes would otherwise serialise on a few LDS words.  Otherwise one
// atomic per lane, except that a wavefront whose active lanes all share one
// digit adds them at once.
template <bool PEERS>
__device__ __forceinline__ void hist_add(uint32_t* h, uint32_t d) {
  const int lane = (int)(threadIdx.x & 63);
  if constexpr (PEERS) {
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint64_t peers = __ballot(1);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    if ((peers & lt) == 0ull) atomicAdd(&h[d], (uint32_t)__popcll(peers));
  } else {
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
    const uint64_t active = __ballot(1);
    if (__ballot(d != d0) == 0ull) {
      if (lane == __ffsll((unsigned long long)active) - 1) atomicAdd(&h[d0], (uint32_t)__popcll(active));
    } else {
      atomicAdd(&h[d], 1u);
    }
  }
}

template <bool PEERS>
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
    for (int u = 0; u < U; ++u) hist_add<PEERS>(h, (k[u] >> shift) & (kRadixBins - 1));
  }
  for (; i < c.end; i += kSortThreads) hist_add<PEERS>(h, (keys[i] >> shift) & (kRadixBins - 1));
  __syncthreads();
  hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's per-block counts.  A
// thread takes kDigitScanItems consecutive counts per round, all loaded before
// any is used, so up to kSortThreads * kDigitScanItems blocks (every plan's
// count) take one round: one load round trip to counts the histogram kernel
// has just written from every XCD, instead of one per 256 blocks.
constexpr int kDigitScanItems = 16;
constexpr int kMaxRadixBlocks = 4096;  // radix blocks per pass, at most (the plans' cap)
static_assert(kSortThreads * kDigitScanItems >= kMaxRadixBlocks, "a digit's scan takes one round");
__global__ __launch_bounds__(kSortThreads) void k_radix_scan_digit(uint32_t* __restrict__ hist, int nb,
                                                                   uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t s_w[4];
  uint32_t* h = hist + (size_t)blockIdx.x * nb;
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += kSortThreads * kDigitScanItems) {
    const int i0 = base + (int)threadIdx.x * kDigitScanItems;
    uint32_t v[kDigitScanItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kDigitScanItems; ++k) {
      v[k] = i0 + k < nb ? h[i0 + k] : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan<uint32_t>(sum, s_w, tot);
#pragma unroll
    for (int k = 0; k < kDigitScanItems; ++k) {
      if (i0 + k < nb) h[i0 + k] = run;
      run += v[k];
    }
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
// which keeps every pass stable.  V is the value type carried with the key.
// With a gather source (the last pass over the compaction indices), the value
// carried out is gather[value in], loaded while the keys are ranked, and only
// the values are written.
constexpr int kItems = 8;
constexpr int kTileKeys = kSortThreads * kItems;
static_assert(kTileKeys == kRadixTile, "block shares are whole tiles");

template <typename V, bool GATHER>
using CarriedT = typename std::conditional<GATHER, Words4, V>::type;  // in registers and LDS
template <typename V, bool GATHER>
using StoredT = typename std::conditional<GATHER, uint4, V>::type;  // in memory

// IOTA: the values carried in are the keys' own input positions (vin is not read).
template <typename V, bool GATHER = false, bool IOTA = false>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                                const V* __restrict__ vin,
                                                                uint32_t* __restrict__ kout,
                                                                StoredT<V, GATHER>* __restrict__ vout,
                                                                const uint32_t* __restrict__ d_count, int shift,
                                                                int nb, const uint32_t* __restrict__ hist,
                                                                const uint32_t* __restrict__ digit_total,
                                                                const uint4* __restrict__ gather) {
  using VO = CarriedT<V, GATHER>;
  __shared__ uint32_t s_keys[kTileKeys];
  __shared__ VO s_vals[kTileKeys];
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
  const Chunk c = chunk_of(count, nb, blockIdx.x);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // item k of lane `lane` in wave w sits at tile offset w*(kItems*64) + k*64 + lane
  const uint32_t o0 = (uint32_t)w * (kItems * 64) + (uint32_t)lane;
  for (uint64_t tb = c.begin; tb < c.end; tb += kTileKeys) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_wc[k][tid] = 0;
    __syncthreads();
    uint32_t key[kItems], rk[kItems];
    V val[kItems];
    VO out[kItems];
    const uint64_t lim = c.end - tb;  // keys left from this tile's start
    {
      // all of the tile's loads first, with indices clamped into the tile and no branch, so they are
      // in flight together rather than one dependent round trip per item
      const uint32_t* kt = kin + tb;
      const V* vt = vin + tb;
      const uint32_t last = (uint32_t)min<uint64_t>(lim, (uint64_t)kTileKeys) - 1;
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const uint32_t o = min(o0 + (uint32_t)k * 64, last);
        key[k] = kt[o];
        if constexpr (IOTA) {
          val[k] = (V)(tb + o);
        } else {
          val[k] = vt[o];
        }
      }
      if constexpr (GATHER) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
          const uint4 g = gather[val[k]];
          out[k] = Words4{g.x, g.y, g.z, g.w};
        }
      } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) out[k] = val[k];
      }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const uint32_t o = o0 + (uint32_t)k * 64;
      const bool valid = o < lim;
      if (!valid) key[k] = 0u;
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
        s_vals[lp] = out[k];
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
        if constexpr (!GATHER) {
          if (kout) kout[g] = kk;  // (no key output: the pass's keys are not needed after it)
        }
        if constexpr (GATHER) {
          const Words4 v = s_vals[i];
          vout[g] = make_uint4(v.x, v.y, v.z, v.w);
        } else {
          vout[g] = s_vals[i];
        }
      }
    }
    __syncthreads();
    s_glob[tid] += tot_d;
  }
}

// ---------------------------------------------------------------------------
// Window binning of the depth-ordered pairs.
//
// Every tile belongs to one binning window of kWinSide x kWinSide tiles.  A
// depth-ordered pair is listed once in every window its tile rect meets (a
// stable LSD radix sort of those (window, item) pairs on the window
// index), so each window's list is in depth order.  A window list is cut into
// chunks of kChunkEntries entries; one wavefront takes a chunk with one lane
// per tile of the window, walks the chunk's entries in order and writes the id
// of every entry that covers its tile to that tile's next output slot.  The
// slots come from the tile's range start plus the counts of the window's
// earlier chunks (k_chunk_counts, k_chunk_scan), so each tile's list is the
// depth order of the pairs covering it, exactly as the stable 64-bit key sort
// orders it, and the incidences themselves are never sorted.
// ---------------------------------------------------------------------------
constexpr int kStepRounds = 8;
constexpr int kStep = kSortThreads * kStepRounds;  // depth-ordered pairs per block step
constexpr int kChunkEntries = 256;                 // window-list entries per chunk (one wavefront)
constexpr int kChunkGroups = kChunkEntries / kWave;
constexpr int kChunkWavesPerBlock = kSortThreads / kWave;

// Per step of kStep depth-ordered entry records: the number of (window, pair)
// items and of (tile, pair) incidences.
__global__ __launch_bounds__(kSortThreads) void k_step_counts(const uint4* __restrict__ ent,
                                                              const uint32_t* __restrict__ d_k,
                                                              uint64_t* __restrict__ step_win,
                                                              uint64_t* __restrict__ step_tiles) {
  __shared__ uint64_t s_w[kSortThreads / 64];
  const uint32_t K = *d_k, nsteps = (K + kStep - 1) / kStep;
  for (uint32_t st = blockIdx.x; st < nsteps; st += gridDim.x) {
    const uint32_t j0 = st * kStep + threadIdx.x;
    uint4 e[kStepRounds];
#pragma unroll
    for (int k = 0; k < kStepRounds; ++k) e[k] = ent[min(j0 + (uint32_t)(k * kSortThreads), K - 1)];
    uint64_t nt = 0, nw = 0;
#pragma unroll
    for (int k = 0; k < kStepRounds; ++k) {
      if (j0 + (uint32_t)(k * kSortThreads) < K) {
        nt += rect_tiles(e[k]);
        nw += rect_windows(e[k]);
      }
    }
    uint64_t tt, tw;
    block_exclusive_scan<uint64_t>(nt, s_w, tt);
    block_exclusive_scan<uint64_t>(nw, s_w, tw);
    if (threadIdx.x == 0) {
      step_tiles[st] = tt;
      step_win[st] = tw;
    }
  }
}

// Exclusive scans of the per-step item and incidence counts in place (one
// block).  M -> d_num_pairs and the overflow flag; the clamped counts for the
// rest of the call are zero on overflow, which makes its kernels no-ops.  A
// thread takes kStepScanItems consecutive steps of both arrays per round (8192
// steps, 16.7 M pairs, per round): at 1024 threads the 64-bit values had
// exceeded the 128 registers a thread may hold and spilled to scratch.
constexpr int kStepScanThreads = 512;
constexpr int kStepScanItems = 16;
__global__ __launch_bounds__(kStepScanThreads) void k_scan_step_counts(uint64_t* __restrict__ step_win,
                                                                   uint64_t* __restrict__ step_tiles,
                                                                   const uint32_t* __restrict__ d_k,
                                                                   uint32_t* __restrict__ d_e,
                                                                   uint32_t* __restrict__ d_m,
                                                                   int64_t* __restrict__ d_pairs,
                                                                   int32_t* __restrict__ d_overflow,
                                                                   int64_t* __restrict__ d_items,
                                                                   uint64_t capacity, int items_bound) {
  __shared__ uint64_t s_w[kStepScanThreads / 64];
  const uint32_t nsteps = (*d_k + kStep - 1) / kStep;
  uint64_t carry_w = 0, carry_t = 0;
  for (uint32_t base = 0; base < nsteps; base += kStepScanThreads * kStepScanItems) {
    const uint32_t i0 = base + threadIdx.x * kStepScanItems;
    uint64_t vw[kStepScanItems], vtl[kStepScanItems], sw = 0, stl = 0;
#pragma unroll
    for (int k = 0; k < kStepScanItems; ++k) {
      vw[k] = i0 + k < nsteps ? step_win[i0 + k] : 0;
      vtl[k] = i0 + k < nsteps ? step_tiles[i0 + k] : 0;
      sw += vw[k];
      stl += vtl[k];
    }
    uint64_t tw, tt;
    uint64_t rw = carry_w + block_exclusive_scan<uint64_t, kStepScanThreads>(sw, s_w, tw);
    uint64_t rt = carry_t + block_exclusive_scan<uint64_t, kStepScanThreads>(stl, s_w, tt);
#pragma unroll
    for (int k = 0; k < kStepScanItems; ++k) {
      if (i0 + k < nsteps) {
        step_win[i0 + k] = rw;
        step_tiles[i0 + k] = rt;
      }
      rw += vw[k];
      rt += vtl[k];
    }
    carry_w += tw;
    carry_t += tt;
  }
  if (threadIdx.x == 0) {
    // the capacity bounds the incidences (tile lists) or the items (window lists)
    const bool over = (items_bound ? carry_w : carry_t) > capacity;
    *d_pairs = (int64_t)carry_t;
    if (d_items) *d_items = (int64_t)carry_w;
    *d_overflow = over ? 1 : 0;
    // with tile lists every item holds at least one incidence, so the item count fits too
    *d_m = over ? 0u : (uint32_t)carry_t;
    *d_e = over ? 0u : (uint32_t)carry_w;
  }
}

// Window item: x = v*N+i, y = its rect clipped to the window, in window tile
// coordinates lx0 | lx1 << 4 | ly0 << 8 | ly1 << 12 (each in [0, 8]).
__device__ inline uint32_t clip_code(uint32_t lo, uint32_t hi, uint32_t w0) {
  // [lo, hi) meets [w0, w0 + kWinSide); the clipped bounds relative to w0
  return (uint32_t)(max(lo, w0) - w0) | ((uint32_t)(min(hi, w0 + kWinSide) - w0) << 4);
}

// The (window, item) pairs in pair order, windows row-major inside a pair:
// key = global window index.
__global__ __launch_bounds__(kSortThreads) void k_window_items(const uint4* __restrict__ ent,
                                                               const uint32_t* __restrict__ d_k,
                                                               const uint32_t* __restrict__ d_e,
                                                               const uint64_t* __restrict__ step_win, ViewTable vt,
                                                               uint32_t n, uint32_t* __restrict__ wkey,
                                                               uint2* __restrict__ witem) {
  __shared__ uint32_t s_w[kSortThreads / 64];
  __shared__ ViewLds s_g;  // win_off, WX
  if (*d_e == 0) return;
  if (threadIdx.x < vt.n_views) {
    s_g.a[threadIdx.x] = vt.v[threadIdx.x].win_off;
    s_g.b[threadIdx.x] = vt.v[threadIdx.x].WX;
  }
  __syncthreads();
  const uint32_t K = *d_k, nsteps = (K + kStep - 1) / kStep;
  for (uint32_t st = blockIdx.x; st < nsteps; st += gridDim.x) {
    const uint32_t j0 = st * kStep + threadIdx.x;
    uint4 e[kStepRounds];
#pragma unroll
    for (int k = 0; k < kStepRounds; ++k) e[k] = ent[min(j0 + (uint32_t)(k * kSortThreads), K - 1)];
    uint64_t o = step_win[st];
#pragma unroll
    for (int k = 0; k < kStepRounds; ++k) {
      const uint32_t nw = (j0 + (uint32_t)(k * kSortThreads) < K) ? rect_windows(e[k]) : 0u;
      uint32_t tot;
      uint64_t p = o + block_exclusive_scan<uint32_t>(nw, s_w, tot);
      o += tot;
      if (nw) {
        const uint32_t v = e[k].z / n, win_off = (uint32_t)s_g.a[v], WX = (uint32_t)s_g.b[v];
        const uint32_t wx0 = (e[k].x & 0xffffu) >> kWinShift, wx1 = (((e[k].x >> 16) - 1) >> kWinShift) + 1;
        const uint32_t wy0 = (e[k].y & 0xffffu) >> kWinShift, wy1 = (((e[k].y >> 16) - 1) >> kWinShift) + 1;
        for (uint32_t wy = wy0; wy < wy1; ++wy) {
          const uint32_t cy = clip_code(e[k].y & 0xffffu, e[k].y >> 16, wy * kWinSide) << 8;
          for (uint32_t wx = wx0; wx < wx1; ++wx, ++p) {
            wkey[p] = win_off + wy * WX + wx;
            witem[p] = make_uint2(e[k].z, cy | clip_code(e[k].x & 0xffffu, e[k].x >> 16, wx * kWinSide));
          }
        }
      }
    }
  }
}

// [wbeg[w], wend[w]) = window w's run in the window-sorted items (both
// pre-filled with 0, so an empty window reads as an empty run).
__global__ void k_window_bounds(const uint32_t* __restrict__ skey, const uint32_t* __restrict__ d_e,
                                uint32_t* __restrict__ wbeg, uint32_t* __restrict__ wend) {
  const uint32_t E = *d_e;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < E; i += gridDim.x * blockDim.x) {
    const uint32_t k = skey[i];
    if (i == 0 || skey[i - 1] != k) wbeg[k] = i;
    if (i + 1 == E || skey[i + 1] != k) wend[k] = i + 1;
  }
}

// cfirst[w] = index of window w's first chunk, cfirst[W] = chunk count (one block).
// With a single pass over the window index (at most 256 windows) that pass's
// digit totals are the windows' item counts: their exclusive scan gives every
// window's run [wbeg, wend) of the sorted items, and a second scan its first
// chunk, with no pass over the sorted keys (one block).
__global__ __launch_bounds__(kScanThreads) void k_window_table(const uint32_t* __restrict__ win_count,
                                                               int n_windows, uint32_t* __restrict__ wbeg,
                                                               uint32_t* __restrict__ wend,
                                                               uint32_t* __restrict__ cfirst,
                                                               uint32_t* __restrict__ d_nchunks) {
  __shared__ uint32_t s_w[kScanThreads / 64];
  uint32_t items = 0, chunks = 0;
  for (int base = 0; base < n_windows; base += kScanThreads) {
    const int w = base + threadIdx.x;
    const uint32_t cnt = w < n_windows ? win_count[w] : 0u;
    const uint32_t nch = (cnt + kChunkEntries - 1) / kChunkEntries;
    uint32_t ti, tc;
    const uint32_t ei = block_exclusive_scan<uint32_t, kScanThreads>(cnt, s_w, ti);
    const uint32_t ec = block_exclusive_scan<uint32_t, kScanThreads>(nch, s_w, tc);
    if (w < n_windows) {
      wbeg[w] = items + ei;
      wend[w] = items + ei + cnt;
      cfirst[w] = chunks + ec;
    }
    items += ti;
    chunks += tc;
  }
  if (threadIdx.x == 0) {
    cfirst[n_windows] = chunks;
    *d_nchunks = chunks;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_chunk_table(const uint32_t* __restrict__ wbeg,
                                                              const uint32_t* __restrict__ wend, int n_windows,
                                                              uint32_t* __restrict__ cfirst,
                                                              uint32_t* __restrict__ d_nchunks) {
  __shared__ uint32_t s_w[kScanThreads / 64];
  uint32_t carry = 0;
  for (int base = 0; base < n_windows; base += kScanThreads) {
    const int w = base + threadIdx.x;
    const uint32_t nch = w < n_windows ? (wend[w] - wbeg[w] + kChunkEntries - 1) / kChunkEntries : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t, kScanThreads>(nch, s_w, tot);
    if (w < n_windows) cfirst[w] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    cfirst[n_windows] = carry;
    *d_nchunks = carry;
  }
}

// Chunk c of the window lists (wave-uniform): its window, its entry run
// [b, e) and the window's view and tile origin.
struct ChunkGeom {
  uint32_t w, b, e;
  int view, tx0, ty0;
};
__device__ inline ChunkGeom chunk_geom(uint32_t c, const uint32_t* __restrict__ cfirst,
                                       const uint32_t* __restrict__ wbeg, const uint32_t* __restrict__ wend,
                                       const ViewTable& vt) {
  // the last window whose first chunk is at or before c (an empty window shares its
  // first-chunk index with the next one, so the search lands on a non-empty window)
  uint32_t lo = 0, hi = (uint32_t)vt.total_windows;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cfirst[mid] <= c) lo = mid;
    else hi = mid;
  }
  ChunkGeom cg;
  cg.w = lo;
  cg.b = wbeg[lo] + (c - cfirst[lo]) * kChunkEntries;
  cg.e = min(cg.b + kChunkEntries, wend[lo]);
  int v = 0;
  for (int u = 1; u < vt.n_views; ++u)
    if ((uint32_t)vt.v[u].win_off <= lo) v = u;
  const ViewGeom& g = vt.v[v];
  const int lw = (int)lo - g.win_off, wy = lw / g.WX;
  cg.view = v;
  cg.tx0 = (lw - wy * g.WX) * kWinSide;
  cg.ty0 = wy * kWinSide;
  return cg;
}

// Chunk visiting order of the chunk kernels: runs of kXcdRun consecutive
// chunks (mostly of one window) go to blocks of one XCD (blocks are handed to
// the kXcds XCDs round robin), so the cache lines shared by neighbouring
// chunks' slot runs of a tile are written through one XCD's L2.  Visit i of
// XCD x is chunk ((i / kXcdRun) * kXcds + x) * kXcdRun + i % kXcdRun, which
// grows with i, and every chunk has exactly one (x, i).
constexpr uint32_t kXcds = 8;
constexpr uint32_t kXcdRun = 16;
__device__ inline uint32_t visited_chunk(uint32_t i, uint32_t xcd) {
  return ((i / kXcdRun) * kXcds + xcd) * kXcdRun + i % kXcdRun;
}

// A chunk's entry records (at most kChunkEntries from b, below e), group q in
// r[q] (lane = entry), loaded with indices clamped into the run and no branch
// so that all of them are in flight at once.
__device__ inline void load_chunk(const uint2* __restrict__ srec, uint32_t b, uint32_t e, int lane,
                                  uint2 (&r)[kChunkGroups]) {
#pragma unroll
  for (int q = 0; q < kChunkGroups; ++q) r[q] = srec[min(b + (uint32_t)(q * kWave + lane), e - 1)];
}

__device__ inline int code_x0(uint32_t c) { return (int)(c & 15u); }
__device__ inline int code_x1(uint32_t c) { return (int)((c >> 4) & 15u); }
__device__ inline int code_y0(uint32_t c) { return (int)((c >> 8) & 15u); }
__device__ inline int code_y1(uint32_t c) { return (int)(c >> 12); }

// Per chunk and tile of its window, the number of the chunk's entries that
// cover the tile: the entries add +1/-1 at the corners of their rects (clipped
// to the window) in a per-wave 8x8 difference grid in LDS, whose 2D inclusive
// prefix is the count; corners in column or row kWinSide lie outside every
// tile of the window and are dropped.  One wavefront per chunk, lane = tile.
__global__ __launch_bounds__(kSortThreads) void k_chunk_counts(const uint2* __restrict__ srec, ViewTable vt,
                                                               const uint32_t* __restrict__ wbeg,
                                                               const uint32_t* __restrict__ wend,
                                                               const uint32_t* __restrict__ cfirst,
                                                               const uint32_t* __restrict__ d_nchunks,
                                                               uint32_t* __restrict__ counts) {
  __shared__ int32_t s_grid[kChunkWavesPerBlock][kWave];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int32_t* grid = s_grid[wv];
  const uint32_t nch = *d_nchunks;
  for (uint32_t c = blockIdx.x * kChunkWavesPerBlock + wv; c < nch; c += gridDim.x * kChunkWavesPerBlock) {
    const ChunkGeom cg = chunk_geom(c, cfirst, wbeg, wend, vt);
    uint2 r[kChunkGroups];
    load_chunk(srec, cg.b, cg.e, lane, r);
    grid[lane] = 0;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < kChunkGroups; ++q) {
      if (cg.b + (uint32_t)(q * kWave + lane) < cg.e) {
        // the rect meets the window (the entry is listed there), so the clipped rect is not empty
        const int lx0 = code_x0(r[q].y), lx1 = code_x1(r[q].y), ly0 = code_y0(r[q].y), ly1 = code_y1(r[q].y);
        atomicAdd(grid + ly0 * kWinSide + lx0, 1);
        if (lx1 < kWinSide) atomicAdd(grid + ly0 * kWinSide + lx1, -1);
        if (ly1 < kWinSide) atomicAdd(grid + ly1 * kWinSide + lx0, -1);
        if (lx1 < kWinSide && ly1 < kWinSide) atomicAdd(grid + ly1 * kWinSide + lx1, 1);
      }
    }
    __builtin_amdgcn_wave_barrier();
    int32_t d = grid[lane];
    // lane = ly * 8 + lx: prefix along the row, then down the column
#pragma unroll
    for (int o = 1; o < kWinSide; o <<= 1) {
      const int32_t y = __shfl_up(d, o, kWinSide);
      if ((lane & (kWinSide - 1)) >= o) d += y;
    }
#pragma unroll
    for (int o = kWinSide; o < kWave; o <<= 1) {
      const int32_t y = __shfl_up(d, o);
      if (lane >= o) d += y;
    }
    counts[(size_t)c * kWave + lane] = (uint32_t)d;
    __builtin_amdgcn_wave_barrier();
  }
}

// One block per window: the counts of the window's chunks become exclusive
// prefixes over the chunks (per tile), and the window's tiles get their
// totals (0 for a window no pair meets).
constexpr int kChunkScanWaves = 16;  // wavefronts per window in the chunk-count scan
constexpr int kChunkScanBatch = 8;   // chunks whose counts a wavefront loads before using them
__global__ __launch_bounds__(kChunkScanWaves * kWave) void k_chunk_scan(const uint32_t* __restrict__ cfirst,
                                                                       ViewTable vt, uint32_t* __restrict__ counts,
                                                                       uint32_t* __restrict__ tile_count) {
  __shared__ uint32_t s_sum[kChunkScanWaves][kWave];
  const uint32_t w = blockIdx.x;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const uint32_t c0 = cfirst[w], c1 = cfirst[w + 1];
  const uint32_t per = (c1 - c0 + kChunkScanWaves - 1) / kChunkScanWaves;
  const uint32_t a = min(c0 + q * per, c1), z = min(a + per, c1);
  // (indices clamped into [a, z): every load is in bounds, the extra ones unused)
  uint32_t sum = 0;
  for (uint32_t cb = a; cb < z; cb += kChunkScanBatch) {
    uint32_t x[kChunkScanBatch];
#pragma unroll
    for (int u = 0; u < kChunkScanBatch; ++u) x[u] = counts[(size_t)min(cb + u, z - 1) * kWave + lane];
#pragma unroll
    for (int u = 0; u < kChunkScanBatch; ++u) sum += cb + u < z ? x[u] : 0u;
  }
  s_sum[q][lane] = sum;
  __syncthreads();
  uint32_t off = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kChunkScanWaves; ++k) {
    const uint32_t s = s_sum[k][lane];
    off += k < q ? s : 0u;
    total += s;
  }
  for (uint32_t cb = a; cb < z; cb += kChunkScanBatch) {
    uint32_t x[kChunkScanBatch];
#pragma unroll
    for (int u = 0; u < kChunkScanBatch; ++u) x[u] = counts[(size_t)min(cb + u, z - 1) * kWave + lane];
#pragma unroll
    for (int u = 0; u < kChunkScanBatch; ++u) {
      if (cb + u < z) {
        counts[(size_t)(cb + u) * kWave + lane] = off;
        off += x[u];
      }
    }
  }
  if (q == 0) {
    int v = 0;
    for (int u = 1; u < vt.n_views; ++u)
      if ((uint32_t)vt.v[u].win_off <= w) v = u;
    const ViewGeom& g = vt.v[v];
    const int lw = (int)w - g.win_off, wy = lw / g.WX;
    const int tx = (lw - wy * g.WX) * kWinSide + (lane & (kWinSide - 1));
    const int ty = wy * kWinSide + (lane >> kWinShift);
    if (tx < g.TX && ty < g.TY) tile_count[g.tile_off + ty * g.TX + tx] = total;
  }
}
__global__ __launch_bounds__(kScanThreads) void k_ranges_from_counts(int total_tiles,
                                                                      const uint32_t* __restrict__ tile_count,
                                                                      const uint32_t* __restrict__ d_m,
                                                                      uint32_t* __restrict__ ranges) {
  __shared__ uint64_t s_w[kScanThreads / 64];
  if (*d_m == 0) {  // no pairs, or the pair capacity overflowed
    for (int t = threadIdx.x; t < total_tiles; t += kScanThreads) ranges[2 * t] = ranges[2 * t + 1] = 0;
    return;
  }
  uint64_t carry = 0;
  for (int base = 0; base < total_tiles; base += kScanThreads * kScanItems) {
    const int t0 = base + (int)threadIdx.x * kScanItems;
    uint32_t cnt[kScanItems];
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      cnt[k] = t0 + k < total_tiles ? tile_count[t0 + k] : 0u;
      sum += cnt[k];
    }
    uint64_t tot;
    uint64_t ex = carry + block_exclusive_scan<uint64_t, kScanThreads>(sum, s_w, tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int t = t0 + k;
      if (t < total_tiles) {
        ranges[2 * t] = cnt[k] ? (uint32_t)ex : 0u;
        ranges[2 * t + 1] = cnt[k] ? (uint32_t)(ex + cnt[k]) : 0u;
      }
      ex += cnt[k];
    }
    carry += tot;
  }
}

// The incidences in their final order: one wavefront per chunk, lane = tile
// of the window, the chunk's entries 64 at a time (group q in r[q], lane =
// entry).  An entry covers tile (lx, ly) exactly when it covers column lx and
// row ly of the window, so 16 ballots (a 64-bit entry mask per column and per
// row) give each tile the mask of the group's entries covering it as
// col[lx] & row[ly].  Each lane expands its mask, in entry order, into an LDS
// stage at its exclusive prefix over the tiles, and the stage leaves with
// consecutive lanes on consecutive slots, so a store instruction writes whole
// runs of tile slots instead of one scattered slot per covered tile.
//
// The grid gives every chunk a wavefront of its own whenever the chunks are
// at most kEmitGridWaves: the vector memory counter is shared by loads and
// stores and completes in order, so a wavefront that loaded its next chunk
// after storing the last one would wait for all of those stores first.
constexpr int kStageSlots = kWave * kWave;  // one group's incidences at most
struct EmitLds {
  uint16_t stage[kStageSlots];  // entry | tile << 6
  uint64_t mask[2 * kWinSide];  // column masks, then row masks
  uint32_t id[kWave];           // the group's entry ids
  uint32_t base[kWave];         // per tile: output slot of stage index 0
};

__global__ __launch_bounds__(kSortThreads) void k_chunk_emit(const uint2* __restrict__ srec,
                                                             const float* __restrict__ rec, ViewTable vt,
                                                             const uint32_t* __restrict__ wbeg,
                                                             const uint32_t* __restrict__ wend,
                                                             const uint32_t* __restrict__ cfirst,
                                                             const uint32_t* __restrict__ d_nchunks,
                                                             const uint32_t* __restrict__ counts,
                                                             const uint32_t* __restrict__ ranges,
                                                             const uint32_t* __restrict__ d_m,
                                                             uint32_t* __restrict__ ids, uint64_t* __restrict__ keys) {
  __shared__ EmitLds s_lds[kChunkWavesPerBlock];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  EmitLds& L = s_lds[wv];
  const int lx = lane & (kWinSide - 1), ly = lane >> kWinShift;
  const uint32_t nch = *d_nchunks, m = *d_m;
  // (the grid is a multiple of kXcds blocks)
  const uint32_t xcd = blockIdx.x % kXcds, stride = (gridDim.x / kXcds) * kChunkWavesPerBlock;
  for (uint32_t i = (blockIdx.x / kXcds) * kChunkWavesPerBlock + wv;; i += stride) {
    const uint32_t c = visited_chunk(i, xcd);
    if (c >= nch) break;
    const ChunkGeom cg = chunk_geom(c, cfirst, wbeg, wend, vt);
    uint2 r[kChunkGroups];
    load_chunk(srec, cg.b, cg.e, lane, r);
    const ViewGeom& g = vt.v[cg.view];
    const uint32_t tx = (uint32_t)(cg.tx0 + lx), ty = (uint32_t)(cg.ty0 + ly);
    // a tile outside the view's grid is never covered (rects are clipped to the grid)
    const bool in_grid = tx < (uint32_t)g.TX && ty < (uint32_t)g.TY;
    const uint32_t tile0 = (uint32_t)g.tile_off + (uint32_t)cg.ty0 * (uint32_t)g.TX + (uint32_t)cg.tx0;
    uint32_t pos = in_grid ? ranges[2 * (tile0 + (uint32_t)ly * (uint32_t)g.TX + (uint32_t)lx)] +
                                 counts[(size_t)c * kWave + lane]
                           : 0u;
    const uint32_t len = cg.e - cg.b;
#pragma unroll
    for (int q = 0; q < kChunkGroups; ++q) {
      if ((uint32_t)(q * kWave) >= len) break;
      const bool valid = (uint32_t)(q * kWave + lane) < len;
      const int lx0 = code_x0(r[q].y), lx1 = code_x1(r[q].y), ly0 = code_y0(r[q].y), ly1 = code_y1(r[q].y);
      uint64_t mine = 0;
#pragma unroll
      for (int j = 0; j < kWinSide; ++j) {
        const uint64_t cm = __ballot(valid && lx0 <= j && j < lx1);
        const uint64_t rm = __ballot(valid && ly0 <= j && j < ly1);
        mine = lane == j ? cm : mine;
        mine = lane == kWinSide + j ? rm : mine;
      }
      if (lane < 2 * kWinSide) L.mask[lane] = mine;
      L.id[lane] = r[q].x;
      __builtin_amdgcn_wave_barrier();
      const uint64_t tm = in_grid ? (L.mask[lx] & L.mask[kWinSide + ly]) : 0ull;
      const uint32_t pop = (uint32_t)__popcll(tm);
      uint32_t incl = pop;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
      }
      const uint32_t pre = incl - pop;
      const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
      L.base[lane] = pos - pre;
      // the mask's halves one after the other, each with 32-bit bit scans
      uint16_t* dst = L.stage + pre;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint32_t mm = (uint32_t)(tm >> (32 * h));
        const uint32_t eh = ((uint32_t)lane << 6) | (uint32_t)(32 * h);
        while (mm) {
          *dst++ = (uint16_t)(eh | (uint32_t)__builtin_ctz(mm));
          mm &= mm - 1u;
        }
      }
      __builtin_amdgcn_wave_barrier();
      for (uint32_t o = (uint32_t)lane; o < total; o += kWave) {
        const uint32_t v = L.stage[o], e = v & 63u, t = v >> 6;
        const uint32_t slot = L.base[t] + o;
        // (the slot bound holds by construction; it keeps every store inside the output)
        if (slot < m) {
          const uint32_t id = L.id[e];
          ids[slot] = id;
          if (keys)
            keys[slot] = ((uint64_t)(tile0 + (t >> kWinShift) * (uint32_t)g.TX + (t & (kWinSide - 1))) << 32) |
                         __float_as_uint(rec[(size_t)id * GS_REC_FLOATS + kDepth]);
        }
      }
      __builtin_amdgcn_wave_barrier();
      pos += pop;
    }
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---------------------------------------------------------------------------
// Workspace layout.
// ---------------------------------------------------------------------------
struct SortPlan {
  uint64_t vn;        // n_views * n
  uint32_t n_seg;     // projection segments (64 Gaussians of one view)
  int nb_seg;         // blocks over the segments
  uint64_t cap;       // pair capacity (bounds the window items too: each holds an incidence)
  int nb_vn;          // radix blocks over the visible pairs
  int nb_items;       // radix blocks over the window items
  int n_steps;        // kStep-pair steps over V*N
  int grid_steps;     // blocks striding over the steps
  int win_passes;     // 8-bit digits of the window index
  uint64_t max_chunks;
  size_t off_counters, off_part_a, off_step_win, off_step_tiles, off_entc, off_ent, off_hist, off_dtot;
  size_t off_akey, off_aval, off_bkey, off_bval, off_wkey0, off_witem0, off_wkey1, off_witem1;
  size_t off_wbeg, off_wend, off_cfirst, off_counts, off_tcount;
  size_t bytes;
};

static SortPlan make_plan(int64_t n, int32_t n_views, int64_t total_tiles, int64_t total_windows,
                          int64_t capacity) {
  SortPlan p;
  p.vn = (uint64_t)n * (uint64_t)n_views;
  p.cap = (uint64_t)capacity;
  p.nb_vn = (int)std::min<uint64_t>(kMaxRadixBlocks, std::max<uint64_t>(1, (p.vn + 2047) / 2048));
  p.n_seg = (uint32_t)((uint64_t)n_views * (((uint64_t)n + 63) / 64));
  p.nb_seg = (int)((p.n_seg + kSortThreads - 1) / kSortThreads);
  p.nb_items = (int)std::min<uint64_t>(kMaxRadixBlocks, std::max<uint64_t>(1, (p.cap + 2047) / 2048));
  p.n_steps = (int)((p.vn + kStep - 1) / kStep);
  p.grid_steps = std::min(p.n_steps, 4096);
  int bits = 1;
  while ((int64_t(1) << bits) < total_windows) ++bits;
  p.win_passes = (bits + kRadixBits - 1) / kRadixBits;
  p.max_chunks = p.cap / kChunkEntries + (uint64_t)total_windows + 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  const uint64_t cap1 = std::max<uint64_t>(p.cap, 1);
  p.off_counters = take(64);
  p.off_part_a = take(sizeof(uint64_t) * p.nb_seg);
  p.off_step_win = take(sizeof(uint64_t) * p.n_steps);
  p.off_step_tiles = take(sizeof(uint64_t) * p.n_steps);
  p.off_entc = take(sizeof(uint4) * p.vn);
  p.off_ent = take(sizeof(uint4) * p.vn);
  p.off_hist = take(sizeof(uint32_t) * kRadixBins * std::max(p.nb_vn, p.nb_items));
  p.off_dtot = take(sizeof(uint32_t) * kRadixBins);
  p.off_akey = take(sizeof(uint32_t) * p.vn);
  p.off_aval = take(sizeof(uint32_t) * p.vn);
  p.off_bkey = take(sizeof(uint32_t) * p.vn);
  p.off_bval = take(sizeof(uint32_t) * p.vn);
  p.off_wkey0 = take(sizeof(uint32_t) * cap1);
  p.off_witem0 = take(sizeof(uint2) * cap1);
  p.off_wkey1 = take(sizeof(uint32_t) * cap1);
  p.off_witem1 = take(sizeof(uint2) * cap1);
  p.off_wbeg = take(sizeof(uint32_t) * (size_t)total_windows);
  p.off_wend = take(sizeof(uint32_t) * (size_t)total_windows);
  p.off_cfirst = take(sizeof(uint32_t) * ((size_t)total_windows + 1));
  p.off_counts = take(sizeof(uint32_t) * kWave * p.max_chunks);
  p.off_tcount = take(sizeof(uint32_t) * (size_t)total_tiles);
  p.bytes = o;
  return p;
}

template <typename V, bool GATHER = false, bool IOTA = false>
static void radix_pass(const uint32_t* kin, const V* vin, uint32_t* kout, StoredT<V, GATHER>* vout,
                       const uint32_t* d_count, int shift, int nb, uint32_t* hist, uint32_t* dtot, hipStream_t st,
                       const uint4* gather = nullptr) {
  // the top digit of the FP32 depth (sign and high exponent bits) takes few distinct values
  if (shift == 24)
    hipLaunchKernelGGL(k_radix_hist<true>, dim3(nb), dim3(kSortThreads), 0, st, kin, d_count, shift, nb, hist);
  else
    hipLaunchKernelGGL(k_radix_hist<false>, dim3(nb), dim3(kSortThreads), 0, st, kin, d_count, shift, nb, hist);
  hipLaunchKernelGGL(k_radix_scan_digit, dim3(kRadixBins), dim3(kSortThreads), 0, st, hist, nb, dtot);
  hipLaunchKernelGGL((k_radix_scatter<V, GATHER, IOTA>), dim3(nb), dim3(kSortThreads), 0, st, kin, vin, kout, vout, d_count,
                     shift, nb, hist, dtot, gather);
}

// Blocks striding over the window-list chunks (a multiple of kXcds).
constexpr int kChunkGrid = 2048;
static_assert(kChunkGrid % kXcds == 0, "chunk grid must split evenly over the XCDs");
// Wavefronts of the emit kernel (a multiple of kXcds blocks): one per chunk up to this many chunks.
constexpr int kEmitGridWaves = 65536;
static_assert((kEmitGridWaves / kChunkWavesPerBlock) % kXcds == 0, "emit grid must split evenly over the XCDs");

// ---------------------------------------------------------------------------
// Spatial order of the Gaussian set (a memory layout, not part of the method):
// the Gaussians sorted by the Z-order (Morton) code of their means.  Each
// kernel that walks the Gaussians in wavefronts of 64 consecutive ones (the
// projection and its backward) then finds a wavefront's splats close together,
// so a view either sees most of them or none, and a wavefront skips the views
// that see none of its Gaussians.
// ---------------------------------------------------------------------------
constexpr int kMortonBits = 10;  // cells per axis: 2^10
constexpr int kBoxThreads = 256;

// Per block: the min and max of x, y, z over its means -> part[6 b .. 6 b + 5] (lo xyz, hi xyz).
__global__ __launch_bounds__(kBoxThreads) void k_box_partial(const float* __restrict__ means, int64_t n,
                                                             float* __restrict__ part) {
  __shared__ float s[6][kBoxThreads / 64];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * kBoxThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBoxThreads) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float m = means[3 * i + a];
      lo[a] = fminf(lo[a], m);
      hi[a] = fmaxf(hi[a], m);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], o));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o));
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      s[a][w] = lo[a];
      s[3 + a][w] = hi[a];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    float v = s[threadIdx.x][0];
    for (int k = 1; k < kBoxThreads / 64; ++k) v = threadIdx.x < 3 ? fminf(v, s[threadIdx.x][k]) : fmaxf(v, s[threadIdx.x][k]);
    part[6 * blockIdx.x + threadIdx.x] = v;
  }
}

// The box over the block partials (one thread per bound) and the Gaussian count for the radix passes.
__global__ void k_box_final(const float* __restrict__ part, int nb, int64_t n, float* __restrict__ box,
                            uint32_t* __restrict__ d_n) {
  const int t = threadIdx.x;
  if (t < 6) {
    float v = part[t];
    for (int b = 1; b < nb; ++b) v = t < 3 ? fminf(v, part[6 * b + t]) : fmaxf(v, part[6 * b + t]);
    box[t] = v;
  }
  if (t == 0) *d_n = (uint32_t)n;
}

// Morton code of each mean: per axis the cell min(2^10 - 1, floor((m - lo) * (2^10 / (hi - lo)))) (a
// degenerate axis gives cell 0; a NaN mean gives cell 0), bits interleaved x0 y0 z0 x1 y1 z1 ...
__device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__global__ __launch_bounds__(kSortThreads) void k_morton(const float* __restrict__ means, int64_t n,
                                                         const float* __restrict__ box, uint32_t* __restrict__ code) {
  uint32_t cell[3];
  const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = box[a], ext = box[3 + a] - lo;
    const float scale = ext > 0.0f ? (float)(1 << kMortonBits) / ext : 0.0f;
    const float q = floorf((means[3 * i + a] - lo) * scale);
    cell[a] = q >= 0.0f ? (uint32_t)fminf(q, (float)((1 << kMortonBits) - 1)) : 0u;  // NaN -> 0
  }
  code[i] = spread3(cell[0]) | (spread3(cell[1]) << 1) | (spread3(cell[2]) << 2);
}

// dst[k * width + c] = src[order[k] * width + c]; an order entry beyond the rows gives NaN rows.
__global__ __launch_bounds__(kSortThreads) void k_gather_rows(const float* __restrict__ src, int64_t n, int width,
                                                              const uint32_t* __restrict__ order,
                                                              float* __restrict__ dst) {
  const int64_t total = n * (int64_t)width;
  for (int64_t e = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kSortThreads) {
    const int64_t k = e / width;
    const int c = (int)(e - k * width);
    const uint32_t o = order[k];
    dst[e] = (int64_t)o < n ? src[(int64_t)o * width + c] : __int_as_float(0x7fc00000);
  }
}

struct OrderPlan {
  int nb_box, nb;
  size_t off_part, off_box, off_n, off_ka, off_kb, off_va, off_vb, off_hist, off_dtot, bytes;
};
static OrderPlan order_plan(int64_t n) {
  OrderPlan p;
  p.nb_box = (int)std::min<int64_t>(1024, (n + kBoxThreads - 1) / kBoxThreads);
  p.nb = (int)std::min<int64_t>(kMaxRadixBlocks, std::max<int64_t>(1, (n + 2047) / 2048));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  p.off_part = take(sizeof(float) * 6 * (size_t)p.nb_box);
  p.off_box = take(sizeof(float) * 6);
  p.off_n = take(sizeof(uint32_t));
  p.off_ka = take(sizeof(uint32_t) * (size_t)n);
  p.off_kb = take(sizeof(uint32_t) * (size_t)n);
  p.off_va = take(sizeof(uint32_t) * (size_t)n);
  p.off_vb = take(sizeof(uint32_t) * (size_t)n);
  p.off_hist = take(sizeof(uint32_t) * kRadixBins * (size_t)p.nb);
  p.off_dtot = take(sizeof(uint32_t) * kRadixBins);
  p.bytes = o;
  return p;
}

}  // namespace gs

extern "C" gs_status gs_spatial_order_workspace_size(int64_t n, size_t* bytes) {
  using namespace gs;
  if (!bytes) return fail(GS_ERR_INVALID_VALUE, "bytes is NULL");
  if (n < 1 || n >= (int64_t(1) << 32) - 1) return fail(GS_ERR_INVALID_VALUE, "n must be in [1, 2^32 - 1)");
  *bytes = order_plan(n).bytes;
  return GS_OK;
}

extern "C" gs_status gs_spatial_order(const float* means, int64_t n, uint32_t* order, void* workspace,
                                      size_t workspace_bytes, void* stream) {
  using namespace gs;
  if (!means || !order) return fail(GS_ERR_INVALID_VALUE, "means and order are required");
  if (n < 1 || n >= (int64_t(1) << 32) - 1) return fail(GS_ERR_INVALID_VALUE, "n must be in [1, 2^32 - 1)");
  const OrderPlan p = order_plan(n);
  if (!workspace || workspace_bytes < p.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(p.bytes) + " bytes");
  hipStream_t st = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  float* part = reinterpret_cast<float*>(ws + p.off_part);
  float* box = reinterpret_cast<float*>(ws + p.off_box);
  uint32_t* d_n = reinterpret_cast<uint32_t*>(ws + p.off_n);
  uint32_t* ka = reinterpret_cast<uint32_t*>(ws + p.off_ka);
  uint32_t* kb = reinterpret_cast<uint32_t*>(ws + p.off_kb);
  uint32_t* va = reinterpret_cast<uint32_t*>(ws + p.off_va);
  uint32_t* vb = reinterpret_cast<uint32_t*>(ws + p.off_vb);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + p.off_hist);
  uint32_t* dtot = reinterpret_cast<uint32_t*>(ws + p.off_dtot);
  hipLaunchKernelGGL(k_box_partial, dim3(p.nb_box), dim3(kBoxThreads), 0, st, means, n, part);
  hipLaunchKernelGGL(k_box_final, dim3(1), dim3(64), 0, st, part, p.nb_box, n, box, d_n);
  hipLaunchKernelGGL(k_morton, dim3((unsigned)((n + kSortThreads - 1) / kSortThreads)), dim3(kSortThreads), 0, st,
                     means, n, box, ka);
  // four stable 8-bit passes over the 30-bit codes, the positions carried as values (ties keep the index order)
  radix_pass<uint32_t, false, true>(ka, nullptr, kb, va, d_n, 0, p.nb, hist, dtot, st);
  radix_pass<uint32_t>(kb, va, ka, vb, d_n, 8, p.nb, hist, dtot, st);
  radix_pass<uint32_t>(ka, vb, kb, va, d_n, 16, p.nb, hist, dtot, st);
  radix_pass<uint32_t>(kb, va, ka, order, d_n, 24, p.nb, hist, dtot, st);
  return check_launch("spatial order");
}

extern "C" gs_status gs_gather_rows(const float* src, int64_t n, int32_t width, const uint32_t* order, float* dst,
                                    void* stream) {
  using namespace gs;
  if (!src || !order || !dst) return fail(GS_ERR_INVALID_VALUE, "src, order and dst are required");
  if (src == dst) return fail(GS_ERR_INVALID_VALUE, "src and dst must not be the same buffer");
  if (n < 1 || n >= (int64_t(1) << 32) - 1 || width < 1 || width > 4096)
    return fail(GS_ERR_INVALID_VALUE, "need n in [1, 2^32 - 1) and width in [1, 4096]");
  const int64_t total = n * (int64_t)width;
  const unsigned grid = (unsigned)std::min<int64_t>(65536, (total + kSortThreads - 1) / kSortThreads);
  hipLaunchKernelGGL(k_gather_rows, dim3(grid), dim3(kSortThreads), 0, as_stream(stream), src, n, width, order, dst);
  return check_launch("gather rows");
}

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
  *bytes = make_plan(n, n_views, vt.total_tiles, vt.total_windows, pair_capacity).bytes;
  return GS_OK;
}

extern "C" gs_status gs_bin_sort(const gs_projected* proj, int64_t n, const gs_camera* cams, int32_t n_views,
                                 const gs_options* opts, const gs_bins* bins, void* workspace, size_t workspace_bytes,
                                 void* stream) {
  using namespace gs;
  gs_status s;
  if ((s = validate_cams(cams, n_views)) != GS_OK) return s;
  if ((s = validate_opts(opts)) != GS_OK) return s;
  if (!proj || !proj->rec || !proj->vis || !proj->vis_count) return fail(GS_ERR_INVALID_VALUE, "proj is incomplete");
  if (reinterpret_cast<uintptr_t>(proj->vis) % 16 != 0) return fail(GS_ERR_INVALID_VALUE, "vis must be 16-byte aligned");
  const bool win_lists = (opts->flags & GS_OPT_WINDOW_LISTS) != 0;
  if (!bins || !bins->d_num_pairs || !bins->d_overflow) return fail(GS_ERR_INVALID_VALUE, "bins is incomplete");
  if (win_lists ? (!bins->items || !bins->win_ranges) : (!bins->ids || !bins->ranges))
    return fail(GS_ERR_INVALID_VALUE, win_lists ? "window lists need bins->items and bins->win_ranges"
                                                : "tile lists need bins->ids and bins->ranges");
  if (win_lists && reinterpret_cast<uintptr_t>(bins->items) % 8 != 0)
    return fail(GS_ERR_INVALID_VALUE, "bins->items must be 8-byte aligned");
  if (n < 1 || (int64_t)n_views * n >= (int64_t(1) << 32) - 1) return fail(GS_ERR_INVALID_VALUE, "bad n");
  if (bins->capacity < 0 || bins->capacity >= (int64_t(1) << 32) - 1)
    return fail(GS_ERR_INVALID_VALUE, "bins->capacity must be in [0, 2^32 - 1)");
  const ViewTable vt = make_view_table(cams, n_views, opts->tile_size);
  const SortPlan p = make_plan(n, n_views, vt.total_tiles, vt.total_windows, bins->capacity);
  if (!workspace || workspace_bytes < p.bytes)
    return fail(GS_ERR_CAPACITY, "workspace too small: need " + std::to_string(p.bytes) + " bytes");
  hipStream_t st = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  uint32_t* counters = reinterpret_cast<uint32_t*>(ws + p.off_counters);
  uint32_t* d_k = counters + 0;        // visible pair count
  uint32_t* d_e = counters + 1;        // window item count (0 on overflow)
  uint32_t* d_m = counters + 2;        // incidence count (0 on overflow)
  uint32_t* d_nchunks = counters + 3;  // window-list chunks
  uint64_t* part_a = reinterpret_cast<uint64_t*>(ws + p.off_part_a);
  uint64_t* step_win = reinterpret_cast<uint64_t*>(ws + p.off_step_win);
  uint64_t* step_tiles = reinterpret_cast<uint64_t*>(ws + p.off_step_tiles);
  uint4* entc = reinterpret_cast<uint4*>(ws + p.off_entc);
  uint4* ent = reinterpret_cast<uint4*>(ws + p.off_ent);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + p.off_hist);
  uint32_t* dtot = reinterpret_cast<uint32_t*>(ws + p.off_dtot);
  uint32_t* akey = reinterpret_cast<uint32_t*>(ws + p.off_akey);
  uint32_t* aval = reinterpret_cast<uint32_t*>(ws + p.off_aval);
  uint32_t* bkey = reinterpret_cast<uint32_t*>(ws + p.off_bkey);
  uint32_t* bval = reinterpret_cast<uint32_t*>(ws + p.off_bval);
  uint32_t* wkey[2] = {reinterpret_cast<uint32_t*>(ws + p.off_wkey0), reinterpret_cast<uint32_t*>(ws + p.off_wkey1)};
  uint2* witem[2] = {reinterpret_cast<uint2*>(ws + p.off_witem0), reinterpret_cast<uint2*>(ws + p.off_witem1)};
  uint32_t* wbeg = reinterpret_cast<uint32_t*>(ws + p.off_wbeg);
  uint32_t* wend = reinterpret_cast<uint32_t*>(ws + p.off_wend);
  uint32_t* cfirst = reinterpret_cast<uint32_t*>(ws + p.off_cfirst);
  uint32_t* counts = reinterpret_cast<uint32_t*>(ws + p.off_counts);
  uint32_t* tcount = reinterpret_cast<uint32_t*>(ws + p.off_tcount);
  const int W = vt.total_windows;

  // 1. visible (view, Gaussian) pairs, compacted in id order with their depth keys and entry records
  const uint4* seg_ent = reinterpret_cast<const uint4*>(proj->vis);
  hipLaunchKernelGGL(k_segment_totals, dim3(p.nb_seg), dim3(kSortThreads), 0, st, proj->vis_count, p.n_seg, part_a);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kSortThreads), 0, st, part_a, p.nb_seg, d_k,
                     (uint64_t)UINT32_MAX);
  hipLaunchKernelGGL(k_compact_segments, dim3(p.nb_seg), dim3(kSortThreads), 0, st, seg_ent, proj->vis_count,
                     p.n_seg, part_a, akey, entc);
  // 2. depth digits (bit 31 of a positive float is 0): four 8-bit passes
  radix_pass<uint32_t, false, true>(akey, nullptr, bkey, bval, d_k, 0, p.nb_vn, hist, dtot, st);
  radix_pass<uint32_t>(bkey, bval, akey, aval, d_k, 8, p.nb_vn, hist, dtot, st);
  radix_pass<uint32_t>(akey, aval, bkey, bval, d_k, 16, p.nb_vn, hist, dtot, st);
  // 3. the last pass carries the entry records (ent[j] = entc[sorted c]); item and incidence counts,
  //    overflow check
  radix_pass<uint32_t, true>(bkey, bval, nullptr, ent, d_k, 24, p.nb_vn, hist, dtot, st, entc);
  hipLaunchKernelGGL(k_step_counts, dim3(p.grid_steps), dim3(kSortThreads), 0, st, ent, d_k, step_win, step_tiles);
  hipLaunchKernelGGL(k_scan_step_counts, dim3(1), dim3(kStepScanThreads), 0, st, step_win, step_tiles, d_k, d_e, d_m,
                     bins->d_num_pairs, bins->d_overflow, bins->d_num_items, p.cap, win_lists ? 1 : 0);
  // 4. (window, item) pairs in depth order, stably sorted on the window index
  hipLaunchKernelGGL(k_window_items, dim3(p.grid_steps), dim3(kSortThreads), 0, st, ent, d_k, d_e, step_win, vt,
                     (uint32_t)n, wkey[0], witem[0]);
  // (window lists: the last pass writes the caller's items)
  uint2* items_out = win_lists ? reinterpret_cast<uint2*>(bins->items) : nullptr;
  // (with a single pass the window runs come from its digit totals, so its keys are not written)
  for (int k = 0; k < p.win_passes; ++k)
    radix_pass<uint2>(wkey[k % 2], witem[k % 2], p.win_passes == 1 ? nullptr : wkey[(k + 1) % 2],
                      (items_out && k + 1 == p.win_passes) ? items_out : witem[(k + 1) % 2], d_e, kRadixBits * k,
                      p.nb_items, hist, dtot, st);
  const uint32_t* skey = wkey[p.win_passes % 2];
  const uint2* srec = items_out ? items_out : witem[p.win_passes % 2];
  if (win_lists) {
    // 5'. the window runs into the caller's win_ranges (begins, then ends); no tile list
    uint32_t* beg = bins->win_ranges;
    uint32_t* end = bins->win_ranges + W;
    if (p.win_passes == 1) {
      hipLaunchKernelGGL(k_window_table, dim3(1), dim3(kScanThreads), 0, st, dtot, W, beg, end, cfirst, d_nchunks);
    } else {
      const unsigned fill_grid = (unsigned)std::min<int64_t>(4096, (2 * W + 255) / 256);
      hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, beg, (uint64_t)2 * W, 0u);
      hipLaunchKernelGGL(k_window_bounds, dim3(p.nb_items), dim3(kSortThreads), 0, st, skey, d_e, beg, end);
    }
    return check_launch("bin/sort");
  }
  // 5. window runs and their chunks
  if (p.win_passes == 1) {
    hipLaunchKernelGGL(k_window_table, dim3(1), dim3(kScanThreads), 0, st, dtot, W, wbeg, wend, cfirst, d_nchunks);
  } else {
    const unsigned fill_grid = (unsigned)std::min<int64_t>(4096, (W + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, wbeg, (uint64_t)W, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, wend, (uint64_t)W, 0u);
    hipLaunchKernelGGL(k_window_bounds, dim3(p.nb_items), dim3(kSortThreads), 0, st, skey, d_e, wbeg, wend);
    hipLaunchKernelGGL(k_chunk_table, dim3(1), dim3(kScanThreads), 0, st, wbeg, wend, W, cfirst, d_nchunks);
  }
  // 6. per-tile counts per chunk, their prefixes over each window's chunks, tile ranges
  hipLaunchKernelGGL(k_chunk_counts, dim3(kChunkGrid), dim3(kSortThreads), 0, st, srec, vt, wbeg, wend, cfirst,
                     d_nchunks, counts);
  hipLaunchKernelGGL(k_chunk_scan, dim3(W), dim3(kChunkScanWaves * kWave), 0, st, cfirst, vt, counts, tcount);
  hipLaunchKernelGGL(k_ranges_from_counts, dim3(1), dim3(kScanThreads), 0, st, vt.total_tiles, tcount, d_m,
                     bins->ranges);
  // 7. the incidences, written in place
  hipLaunchKernelGGL(k_chunk_emit, dim3(kEmitGridWaves / kChunkWavesPerBlock), dim3(kSortThreads), 0, st, srec,
                     proj->rec, vt,
                     wbeg, wend, cfirst, d_nchunks, counts, bins->ranges, d_m, bins->ids, bins->keys);
  return check_launch("bin/sort");
}
