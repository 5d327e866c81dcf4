// Stable LSD radix sort of (key, index) pairs (Section 3.2 sorts key/index
// pairs with a device-wide radix sort), segmented: every segment is sorted
// on its own, in place, and a plain sort is the one-segment case.
//
// Design (one histogram pass, then one scatter pass per digit):
//  * segment descriptors live in device memory, so sizes can come from the
//    device (a compaction count, a batch table) and one captured launch
//    sequence serves any mix;
//  * k_seg_hist reads every key once and builds the digit histograms of all
//    passes per segment (a single sort spreads them over one copy per XCD,
//    so that few atomics meet on one device word, and a block counts into
//    eight LDS copies, so that lanes with equal digits seldom meet on one
//    LDS word); for the fused call's dense sort, k_keys_hist computes the
//    keys from the rays and counts them in the same pass instead;
//  * k_seg_pass blocks (512 threads) are persistent.  A sort that has the
//    device to itself takes tiles in a fixed order (round r of G tiles:
//    runs of 16 consecutive tiles dealt to the XCDs in turn, so that the
//    seams between neighbouring tiles' digit runs meet in one L2), so no
//    shared tile counter is contended; the batched layer,
//    whose sorts may share the device with other kernels, by default takes
//    them in order from an atomic counter, so that a tile is only ever held
//    by a running block (each block takes its next ticket while it works on
//    the current tile).  A tile is ranked by digit with wave64 ballots (a match over the
//    digit's bits gives each lane its peers; the lowest peer adds the group's
//    size to the wave's digit count with one LDS atomic), its digit counts
//    are published, the previous tiles of the same segment are looked back
//    for the global offsets (decoupled look-back, Merrill and Garland 2016),
//    and the tile is reordered in LDS and written as contiguous digit runs
//    (the last pass of the fused call also moves the rays to their slots).
//  * The look-back is two-level: tiles form groups of kGroup, and the last
//    tile of a group also publishes the group's total and then its inclusive
//    prefix, so a tile reads its own group's tiles and then whole groups,
//    kGroup tiles per word.  Every round reads its whole window for each
//    digit, past the L2, so the windows are kept small.
//  * Waits never depend on other blocks being resident: an entry that stays
//    unpublished for a bounded number of polls is computed by the waiting
//    thread itself from the input keys (the fallback of decoupled look-back,
//    Smith, Levien and Owens 2024), so every wait ends.  With tiles from the
//    counter every awaited tile is held by a running block, so the bound is
//    set far out and only guards against the unexpected.
// Ranking keeps input order within a digit, so the sort is stable and the
// output is the unique (key, index) lexicographic order for ascending input
// indices.
#include <algorithm>
#include <utility>

#include "common.hpp"
#include "keys_dev.hpp"
#include "sort_seg.hpp"
#include "wave.hpp"

namespace rr {
namespace {

constexpr int kSortThreads = 512;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr uint32_t kGroup = 8;           // tiles per look-back group
constexpr uint32_t kTileRun = 16;        // consecutive tiles of one XCD in the fixed tile order
// Words read per look-back round.  Every word is a load past the L2, and
// their number costs more than the rounds: windows of 4 sorted 64M pairs
// 6% faster than windows of 7 and 8, and 2, 3 or 4 with 8 were slower.
constexpr uint32_t kTileWindow = 4;   // tile words
constexpr uint32_t kGroupWindow = 4;  // group words
constexpr uint32_t kFallbackSpins = 128;       // polls of an unpublished entry before computing it
constexpr uint32_t kFallbackSpinsCounted = 1u << 16;  // tiles from the counter: waiting is always safe
constexpr uint32_t kHistUnit = 4096;  // keys per histogram work unit (8 per thread)
// Buckets of the most-significant-digit sort of at most kWaveCap keys can
// each be sorted by one wave (k_msd_wave): when every bucket is that small,
// k_msd_wave sorts them all and k_msd_local has nothing to do, else
// k_msd_local sorts them all.
constexpr uint32_t kWaveCap = 512;
constexpr uint32_t kHistCopies = 8;   // histogram copies of a single-segment sort (one per XCD)
constexpr uint32_t kHistLaneCopies = 8;  // LDS histogram copies per block, lane l counts into copy l % 8
constexpr uint32_t kHistCopyPad = 8;     // words between LDS copies beyond their size: copy c starts 8c banks on

// Exclusive scan of one value per thread over the block (wave shuffles,
// then the kSortWaves wave totals); s needs kSortWaves words.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* s, uint32_t* total) {
  const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == kWave - 1) s[wave] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) {
    const uint32_t t = s[w];
    pre += (uint32_t)w < wave ? t : 0u;
    tot += t;
  }
  *total = tot;
  __syncthreads();
  return pre + x - v;
}

// Segment holding global tile t (segments ordered by tile_off).
__device__ __forceinline__ uint32_t seg_of_tile(const SortSeg* segs, uint32_t nseg, uint32_t t) {
  uint32_t lo = 0, hi = nseg;  // invariant: segs[lo].tile_off <= t
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (segs[mid].tile_off <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One segment of n = min(*count_dev, n_max) keys; clears its histograms
// (all copies, spread over the blocks).
__global__ void k_seg_setup_single(const uint32_t* count_dev, uint32_t n_max, uint32_t tile, SortHdr* hdr,
                                   SortSeg* segs, uint32_t* __restrict__ hist, uint32_t hist_words,
                                   uint32_t* __restrict__ counters, uint32_t n_counters) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < hist_words; i += gridDim.x * blockDim.x) hist[i] = 0;
  if (blockIdx.x != 0) return;
  if (threadIdx.x == 0) {
    uint32_t n = n_max;
    if (count_dev) n = min(*count_dev, n_max);
    const uint32_t tiles = (n + tile - 1) / tile;
    segs[0] = SortSeg{0u, n, 0u, tiles};
    *hdr = SortHdr{1u, tiles, n, 0u};
  }
  for (uint32_t i = threadIdx.x; i < n_counters; i += blockDim.x) counters[i] = 0;
}

// Clears the histograms of a segment table set up by the caller, and the
// tile counters.
__global__ void k_seg_init(const SortHdr* hdr, uint32_t* __restrict__ hist, uint32_t words_per_seg,
                           uint32_t* __restrict__ counters, uint32_t n_counters) {
  const uint32_t n = hdr->nseg * words_per_seg;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) hist[i] = 0;
  if (blockIdx.x == 0)
    for (uint32_t i = threadIdx.x; i < n_counters; i += blockDim.x) counters[i] = 0;
}

// The single segment of the most-significant-digit sort (n = min(*count_dev,
// n_max) keys): clears the digit histograms and the (dh, dl) bucket sizes,
// and empties the second pass's header, which its first pass fills when
// there are keys.
__global__ void k_msd_setup(const uint32_t* count_dev, uint32_t n_max, uint32_t tile, SortHdr* hdr, SortSeg* segs,
                            uint32_t* __restrict__ hist, uint32_t hist_words, uint32_t* __restrict__ hist2,
                            uint32_t hist2_words, SortHdr* hdr2, MsdPlan* plan) {
  const uint32_t stride = gridDim.x * blockDim.x, gid = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t i = gid; i < hist_words; i += stride) hist[i] = 0;
  for (uint32_t i = gid; i < hist2_words; i += stride) hist2[i] = 0;
  if (gid == 0) {
    uint32_t n = n_max;
    if (count_dev) n = min(*count_dev, n_max);
    const uint32_t tiles = (n + tile - 1) / tile;
    segs[0] = SortSeg{0u, n, 0u, tiles};
    *hdr = SortHdr{1u, tiles, n, 0u};
    *hdr2 = SortHdr{0u, 0u, 0u, 0u};
    *plan = MsdPlan{1u, 0u, 0u, 0u};  // no bucket larger than kWaveCap yet
  }
}

// Digit histograms of every pass per segment.  Blocks take contiguous runs
// of kHistUnit-key units (a unit never straddles a segment), load a unit's
// keys before counting them, and flush their LDS counts when the segment
// changes, block b into histogram copy b % copies (blocks are dealt to the
// XCDs in turn, so with 8 copies each copy takes the atomics of one XCD and
// no device word takes more than about blocks / copies of them); the
// look-back words (tile and group) the passes will use are cleared too.
// Neighbouring rays of a coherent wavefront share their high digits, and the
// LDS atomics of lanes that hit one word serialize: each lane therefore
// counts into one of kHistLaneCopies copies (lane mod 8), laid out so that
// the copies of a word sit in different banks, and the copies are summed at
// the flush.
// Adds the block's lane-copy counts of the first `words` histogram words to
// dst (device atomics, zero counts skipped) and clears them for reuse.  The
// caller synchronises the block before and, to reuse s_h, after.
__device__ __forceinline__ void flush_lane_hist(uint32_t* s_h, uint32_t stride, uint32_t words,
                                                uint32_t* __restrict__ dst) {
  for (uint32_t i = threadIdx.x; i < words; i += kSortThreads) {
    uint32_t v = 0;
#pragma unroll
    for (uint32_t c = 0; c < kHistLaneCopies; ++c) {
      v += s_h[c * stride + i];
      s_h[c * stride + i] = 0;
    }
    if (v) atomicAdd(&dst[i], v);
  }
}

// Clears the look-back words of `tiles` tiles and `groups` groups of every
// pass, spread over the grid.
__device__ __forceinline__ void clear_lookback(uint32_t* __restrict__ status, uint32_t status_pass_stride,
                                               uint32_t tiles, uint32_t* __restrict__ gstatus,
                                               uint32_t gstatus_pass_stride, uint32_t groups, uint32_t passes,
                                               uint32_t R) {
  const uint32_t stride = gridDim.x * kSortThreads;
  for (uint32_t p = 0; p < passes; ++p) {
    for (uint32_t i = blockIdx.x * kSortThreads + threadIdx.x; i < tiles * R; i += stride)
      status[(size_t)p * status_pass_stride + i] = 0;
    for (uint32_t i = blockIdx.x * kSortThreads + threadIdx.x; i < groups * R; i += stride)
      gstatus[(size_t)p * gstatus_pass_stride + i] = 0;
  }
}

// With a plan (the second pass of the most-significant-digit sort) only
// digit plan->dl is counted, as the histogram of pass 0.  The look-back
// words of clear_passes passes are cleared for the segments' tiles plus
// extra_tiles, and their groups plus extra_groups.
template <typename K, int DB, int KPT>
__global__ __launch_bounds__(kSortThreads) void k_seg_hist(const K* __restrict__ keys, const SortHdr* hdr,
                                                           const SortSeg* __restrict__ segs, uint32_t passes,
                                                           uint32_t copies, uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ status,
                                                           uint32_t status_pass_stride,
                                                           uint32_t* __restrict__ gstatus,
                                                           uint32_t gstatus_pass_stride, const MsdPlan* plan,
                                                           uint32_t clear_passes, uint32_t extra_tiles,
                                                           uint32_t extra_groups) {
  constexpr uint32_t R = 1u << DB;
  constexpr uint32_t kTile = kSortThreads * KPT;
  constexpr uint32_t kUnitsPerTile = kTile >= kHistUnit ? kTile / kHistUnit : 1u;
  constexpr uint32_t kUnitKeys = kTile >= kHistUnit ? kHistUnit : kTile;
  constexpr uint32_t kPer = kUnitKeys / kSortThreads;
  constexpr uint32_t kMaxPasses = (8 * sizeof(K) + DB - 1) / DB;
  static_assert(kHistUnit % kSortThreads == 0, "unit size");
  constexpr uint32_t kStride = kMaxPasses * R + kHistCopyPad;
  __shared__ uint32_t s_h[kHistLaneCopies * kStride];
  const uint32_t nseg = hdr->nseg, T = hdr->total_tiles;
  const uint32_t U = T * kUnitsPerTile;
  const uint32_t words = passes * R;
  const uint32_t copy = blockIdx.x % copies;
  const uint32_t shift0 = plan ? plan->dl * DB : 0u;  // digit of pass 0
  uint32_t* const lane_h = s_h + (threadIdx.x % kHistLaneCopies) * kStride;
  for (uint32_t i = threadIdx.x; i < kHistLaneCopies * kStride; i += kSortThreads) s_h[i] = 0;
  __syncthreads();
  const uint32_t u0 = (uint32_t)(((uint64_t)blockIdx.x * U) / gridDim.x);
  const uint32_t u1 = (uint32_t)(((uint64_t)(blockIdx.x + 1) * U) / gridDim.x);
  uint32_t cur = u0 < u1 ? seg_of_tile(segs, nseg, u0 / kUnitsPerTile) : 0u;
  for (uint32_t u = u0; u < u1; ++u) {
    const uint32_t t = u / kUnitsPerTile;
    uint32_t s = cur;
    while (s + 1 < nseg && segs[s + 1].tile_off <= t) ++s;  // block-uniform
    if (s != cur) {
      __syncthreads();
      flush_lane_hist(s_h, kStride, words, hist + ((size_t)cur * copies + copy) * words);
      __syncthreads();
      cur = s;
    }
    const SortSeg sg = segs[s];
    const uint32_t first = sg.off + (t - sg.tile_off) * kTile + (u % kUnitsPerTile) * kUnitKeys;
    const uint32_t last = sg.off + sg.n;
    K k[kPer];
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint32_t i = first + q * kSortThreads + threadIdx.x;
      k[q] = i < last ? keys[i] : (K)0;
    }
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      if (first + q * kSortThreads + threadIdx.x >= last) continue;
      for (uint32_t p = 0; p < passes; ++p)
        atomicAdd(&lane_h[p * R + ((uint32_t)(k[q] >> (shift0 + p * DB)) & (R - 1))], 1u);
    }
  }
  __syncthreads();
  if (u0 < u1) flush_lane_hist(s_h, kStride, words, hist + ((size_t)cur * copies + copy) * words);
  // clear the look-back words of the tiles and groups the passes will use
  if (clear_passes)
    clear_lookback(status, status_pass_stride, T + extra_tiles, gstatus, gstatus_pass_stride,
                   (T + extra_tiles) / kGroup + nseg + extra_groups, clear_passes, R);
}

// The keys of a dense single-segment sort computed and counted in one pass
// (the fused reorder-and-trace call): block b takes a contiguous run of
// kHistUnit-ray units, computes each ray's key exactly as the keys kernel
// does (key and identity index written out), counts the 8-bit digits of
// every pass into the lane copies in LDS and flushes them into histogram
// copy b % copies like k_seg_hist, and clears the look-back words of
// status_tiles tiles and status_groups groups per pass.  The histogram
// copies must have been cleared before.
template <int KIND, typename K>
__global__ __launch_bounds__(kSortThreads) void k_keys_hist(const float4* __restrict__ rays, uint32_t n,
                                                            KeyPlan P, K* __restrict__ keys,
                                                            uint32_t* __restrict__ idx, uint32_t passes,
                                                            uint32_t copies, uint32_t* __restrict__ hist,
                                                            uint32_t* __restrict__ status,
                                                            uint32_t status_pass_stride, uint32_t status_tiles,
                                                            uint32_t* __restrict__ gstatus,
                                                            uint32_t gstatus_pass_stride, uint32_t status_groups,
                                                            uint32_t clear_passes) {
  constexpr int DB = 8;
  constexpr uint32_t R = 1u << DB;
  constexpr uint32_t kPer = kHistUnit / kSortThreads;
  constexpr uint32_t kMaxPasses = 8 * sizeof(K) / DB;
  constexpr uint32_t kStride = kMaxPasses * R + kHistCopyPad;
  __shared__ uint32_t s_h[kHistLaneCopies * kStride];
  const uint32_t words = passes * R;
  const uint32_t copy = blockIdx.x % copies;
  uint32_t* const lane_h = s_h + (threadIdx.x % kHistLaneCopies) * kStride;
  for (uint32_t i = threadIdx.x; i < kHistLaneCopies * kStride; i += kSortThreads) s_h[i] = 0;
  __syncthreads();
  const uint32_t U = (n + kHistUnit - 1) / kHistUnit;
  const uint32_t u0 = (uint32_t)(((uint64_t)blockIdx.x * U) / gridDim.x);
  const uint32_t u1 = (uint32_t)(((uint64_t)(blockIdx.x + 1) * U) / gridDim.x);
  for (uint32_t u = u0; u < u1; ++u) {
    const uint32_t first = u * kHistUnit;
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint32_t i = first + q * kSortThreads + threadIdx.x;
      if (i >= n) continue;
      const float4 a = rays[2 * (size_t)i];
      const float4 b = rays[2 * (size_t)i + 1];
      const K k = (K)ray_key<KIND>(a, b, P, i);
      keys[i] = k;
      idx[i] = i;
      for (uint32_t p = 0; p < passes; ++p)
        atomicAdd(&lane_h[p * R + ((uint32_t)(k >> (p * DB)) & (R - 1))], 1u);
    }
  }
  __syncthreads();
  if (u0 < u1) flush_lane_hist(s_h, kStride, words, hist + (size_t)copy * words);
  clear_lookback(status, status_pass_stride, status_tiles, gstatus, gstatus_pass_stride, status_groups, clear_passes,
                 R);
}

template <typename K, int DB, int KPT>
struct PassSmem {
  static constexpr uint32_t R = 1u << DB;
  static constexpr uint32_t kTile = kSortThreads * KPT;
  K keys[kTile];
  uint32_t idx[kTile];
  uint32_t wave_hist[kSortWaves][R];  // per-wave digit counts, then their tile positions
  uint32_t delta[R];                  // output position minus tile position, per digit
  uint32_t base[R];
  uint32_t scan[kSortWaves];
  uint32_t ticket;  // next tile, when tiles come from a counter
  uint32_t nonuni;  // digits in which the keys differ (the first pass of the MSD sort)
};

// The two scatter passes of the most-significant-digit sort; mode 0 is a
// pass of the LSD sort.  Mode 1, the first pass of a single-segment sort:
// every block picks the digits itself from the histograms and the first key
// (digit d is the same in every key exactly when the first key's digit-d
// value counts all keys): dh is the highest digit that differs, dl the next
// one below it (another digit when none below differs); the pass scatters by
// dh, and the block holding tile 0 writes the plan and the 256 segments of
// the second pass, one per value of dh.  Mode 2, the second pass: scatters
// each of those segments by digit dl and records where every (dh, dl)
// bucket starts.
struct MsdArgs {
  uint32_t mode;
  MsdPlan* plan;
  SortHdr* hdr2;
  SortSeg* segs2;
  uint32_t* bstart;
};

__device__ __forceinline__ uint32_t load_status(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_status(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Number of keys with digit d in local tile lt of segment sg, counted from
// the input: what that tile's owner publishes, for the look-back fallback.
template <typename K, uint32_t kTile>
__device__ __noinline__ uint32_t count_digit(const K* __restrict__ keys_in, SortSeg sg, uint32_t lt, uint32_t shift,
                                             uint32_t mask, uint32_t d) {
  const uint32_t first = sg.off + lt * kTile;
  const uint32_t n = min(kTile, sg.n - lt * kTile);
  uint32_t c = 0;
  for (uint32_t i = 0; i < n; ++i) c += ((uint32_t)(keys_in[first + i] >> shift) & mask) == d ? 1u : 0u;
  return c;
}

// Published value of local tile lt for digit d, waiting for it at most
// `fallback` polls and counting it from the input after that.
template <typename K, uint32_t kTile>
__device__ uint32_t tile_word(const uint32_t* status, const K* __restrict__ keys_in, SortSeg sg, uint32_t lt,
                              uint32_t R, uint32_t shift, uint32_t d, uint32_t fallback) {
  for (uint32_t spins = 0; spins < fallback; ++spins) {
    const uint32_t w = load_status(&status[(size_t)(sg.tile_off + lt) * R + d]);
    if (w & ~kStatusCountMask) return w;
    __builtin_amdgcn_s_sleep(2);
  }
  return kStatusAggregate | count_digit<K, kTile>(keys_in, sg, lt, shift, R - 1, d);
}

// Exclusive prefix of digit d before local tile lt (lt > 0) of segment sg,
// whose own count is c.  Phase A sums the published words of the earlier
// tiles of lt's group, nearest first, up to an inclusive one; phase B
// continues over whole groups.  A group word still unpublished after the
// wait limit is replaced by its tiles' words, and a tile word by a count
// from the input.  The last tile of a group passes its group word as gword:
// when phase A ends without an inclusive word, the group total is published
// there before phase B.
template <typename K, uint32_t kTile>
__device__ uint32_t look_back(const uint32_t* status, const uint32_t* gstatus, const K* __restrict__ keys_in,
                              SortSeg sg, uint32_t gbase, uint32_t lt, uint32_t R, uint32_t shift, uint32_t d,
                              uint32_t c, uint32_t* gword, uint32_t fallback) {
  const uint32_t g = lt / kGroup, gs = g * kGroup;
  uint32_t acc = 0;
  bool done = false;
  uint32_t spins = 0;
  int32_t j = (int32_t)lt - 1;  // nearest tile not yet accounted for
  while (!done && j >= (int32_t)gs) {
    const int32_t lim = j - (int32_t)gs + 1;  // valid entries in the window
    uint32_t w[kTileWindow];
#pragma unroll
    for (int q = 0; q < (int)kTileWindow; ++q)
      w[q] = q < lim ? load_status(&status[(size_t)(sg.tile_off + j - q) * R + d]) : 0u;
    uint32_t a = 0;
    int used = 0;
    bool blocked = false;
#pragma unroll
    for (int q = 0; q < (int)kTileWindow; ++q) {
      if (done || blocked || q >= lim) continue;
      const uint32_t flag = w[q] & ~kStatusCountMask;
      if (flag == 0) {
        blocked = true;
      } else {
        a += w[q] & kStatusCountMask;
        ++used;
        if (flag == kStatusPrefix) done = true;
      }
    }
    acc += a;
    j -= used;
    if (blocked) {
      if (++spins >= fallback) {
        acc += count_digit<K, kTile>(keys_in, sg, (uint32_t)j, shift, R - 1, d);
        --j;
        spins = 0;
      } else {
        __builtin_amdgcn_s_sleep(2);
      }
    }
  }
  if (gword && !done) store_status(gword, kStatusAggregate | (acc + c));
  int32_t G = (int32_t)g - 1;  // nearest group not yet accounted for
  spins = 0;
  while (!done && G >= 0) {
    const int32_t lim = G + 1;
    uint32_t w[kGroupWindow];
#pragma unroll
    for (int q = 0; q < (int)kGroupWindow; ++q)
      w[q] = q < lim ? load_status(&gstatus[(size_t)(gbase + G - q) * R + d]) : 0u;
    uint32_t a = 0;
    int used = 0;
    bool blocked = false;
#pragma unroll
    for (int q = 0; q < (int)kGroupWindow; ++q) {
      if (done || blocked || q >= lim) continue;
      const uint32_t flag = w[q] & ~kStatusCountMask;
      if (flag == 0) {
        blocked = true;
      } else {
        a += w[q] & kStatusCountMask;
        ++used;
        if (flag == kStatusPrefix) done = true;
      }
    }
    acc += a;
    G -= used;
    if (blocked) {
      if (++spins >= fallback) {
        // the group's last tile has not published: read its tiles instead
        for (int32_t t = G * (int32_t)kGroup + (int32_t)kGroup - 1; t >= G * (int32_t)kGroup && !done; --t) {
          const uint32_t v = tile_word<K, kTile>(status, keys_in, sg, (uint32_t)t, R, shift, d, fallback);
          acc += v & kStatusCountMask;
          if ((v & ~kStatusCountMask) == kStatusPrefix) done = true;
        }
        --G;
        spins = 0;
      } else {
        __builtin_amdgcn_s_sleep(2);
      }
    }
  }
  return acc;
}

template <typename K, int DB, int KPT, int MODE = 0>
__global__ __launch_bounds__(kSortThreads) void k_seg_pass(const K* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ idx_in,
                                                           K* __restrict__ keys_out, uint32_t* __restrict__ idx_out,
                                                           const SortHdr* hdr, const SortSeg* __restrict__ segs,
                                                           uint32_t shift_in, uint32_t passes, uint32_t pass_in,
                                                           uint32_t copies, const uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ status,
                                                           uint32_t* __restrict__ gstatus,
                                                           uint32_t* tile_counter,
                                                           const float4* __restrict__ gather_in,
                                                           float4* __restrict__ gather_out, uint32_t gather_n,
                                                           MsdArgs msd) {
  using S = PassSmem<K, DB, KPT>;
  constexpr uint32_t R = S::R;
  constexpr uint32_t kTile = S::kTile;
  __shared__ S sm;
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const uint32_t nseg = hdr->nseg, T = hdr->total_tiles;
  const SortSeg seg0 = segs[0];  // loaded beside the header: a single sort needs no other
  uint32_t cur = 0xFFFFFFFFu;  // segment whose digit bases are in sm.base

  for (uint32_t i = tid; i < kSortWaves * R; i += kSortThreads) (&sm.wave_hist[0][0])[i] = 0;

  uint32_t shift = shift_in, pass = pass_in, dh = 0, dl = 0;
  if constexpr (MODE == 1) {
    if (tid == 0) sm.nonuni = 0;
    __syncthreads();
    const uint32_t n_all = hdr->total_keys;
    if (tid < passes && n_all > 0) {
      const uint32_t dg = (uint32_t)(keys_in[seg0.off] >> (tid * DB)) & (R - 1);
      uint32_t c = 0;
      for (uint32_t cc = 0; cc < copies; ++cc) c += hist[((size_t)cc * passes + tid) * R + dg];
      if (c != n_all) atomicOr(&sm.nonuni, 1u << tid);
    }
    __syncthreads();
    const uint32_t m = sm.nonuni;
    dh = m ? 31u - (uint32_t)__builtin_clz(m) : passes - 1;
    const uint32_t below = m & ((1u << dh) - 1u);
    dl = below ? 31u - (uint32_t)__builtin_clz(below) : (dh > 0 ? dh - 1 : 1u);
    shift = dh * DB;
    pass = dh;
  } else if constexpr (MODE == 2) {
    shift = msd.plan->dl * DB;
  }

  // Keys and indices of a tile, loaded wave-striped: wave w owns KPT
  // consecutive groups of 64.  The next tile's loads are issued before the
  // current tile is written out, so their latency overlaps the writes.
  K k[KPT];
  uint32_t v[KPT];
  uint32_t rank[KPT];
  auto load_tile = [&](uint32_t base, uint32_t tile_n) {
    const K* kb = keys_in + base;  // block-uniform tile start
    const uint32_t* ib = idx_in + base;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const uint32_t pos = wave * (KPT * kWave) + j * kWave + lane;
      const bool ok = pos < tile_n;
      k[j] = ok ? kb[pos] : (K)0;
      v[j] = ok ? ib[pos] : 0u;
    }
  };
  // tiles in a fixed order, or in order from the counter (tile_counter).
  // The fixed order is XCD-aware: workgroups go to the XCDs round-robin, so
  // block b would take tile b and neighbouring tiles would sit on different
  // XCDs.  Instead every round of gridDim.x tiles is cut into runs of
  // kTileRun consecutive tiles, dealt to the XCDs in turn.  A digit's run
  // from tile t ends where tile t + 1's run of that digit starts, so within
  // a tile run the partial cache lines at those seams meet in one L2 before
  // they are written back.  The runs are short, so the tiles in flight stay
  // a narrow window and look-backs find their predecessors started.
  // Blocks past the last whole span of kXcds runs keep tile = block.
  const bool counted = tile_counter != nullptr;
  if (counted) {
    if (tid == 0) sm.ticket = atomicAdd(tile_counter, 1u);
    __syncthreads();
  }
  uint32_t tile = blockIdx.x;
  if (counted) {
    tile = sm.ticket;
  } else if (blockIdx.x < gridDim.x / (kXcds * kTileRun) * (kXcds * kTileRun)) {
    const uint32_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    tile = j / kTileRun * (kXcds * kTileRun) + x * kTileRun + j % kTileRun;
  }
  uint32_t s = 0;
  SortSeg sg{};
  if (tile < T) {
    s = nseg == 1 ? 0u : seg_of_tile(segs, nseg, tile);
    sg = nseg == 1 ? seg0 : segs[s];
    const uint32_t lt = tile - sg.tile_off;
    load_tile(sg.off + lt * kTile, min(kTile, sg.n - lt * kTile));
  }
  while (tile < T) {  // block-uniform
    const uint32_t lt = tile - sg.tile_off;
    const uint32_t tile_n = min(kTile, sg.n - lt * kTile);
    __syncthreads();  // the previous tile's LDS reads are done; wave_hist is clear
    if (counted && tid == 0) sm.ticket = atomicAdd(tile_counter, 1u);  // read after the reorder barrier

    // ---- rank within the wave, in (j, lane) order.  The lowest lane of
    // each group of equal digits adds the group's size to the wave's count
    // with an LDS atomic (the leaders of one step hold distinct digits, and
    // a wave's LDS operations take effect in order), and the group's lanes
    // take the count it returned once every step has been issued.
    uint32_t old[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const uint32_t pos = wave * (KPT * kWave) + j * kWave + lane;
      const bool ok = pos < tile_n;
      const uint32_t d = (uint32_t)(k[j] >> shift) & (R - 1);
      const uint64_t peers = match_digit<DB>(d, __ballot(ok));
      const uint32_t leader = ok ? (uint32_t)__builtin_ctzll(peers) : lane;
      rank[j] = lanes_below(peers) | (leader << 16);
      old[j] = 0;
      if (ok && lane == leader) old[j] = atomicAdd(&sm.wave_hist[wave][d], (uint32_t)__popcll(peers));
    }
#pragma unroll
    for (int j = 0; j < KPT; ++j) rank[j] = (rank[j] & 0xFFFFu) + __shfl(old[j], (int)(rank[j] >> 16), kWave);
    __syncthreads();

    // ---- digit bases of this segment and pass: offset + exclusive prefix
    if (s != cur) {  // block-uniform
      uint32_t total;
      uint32_t h = 0;
      if (tid < R)
        for (uint32_t c = 0; c < copies; ++c) h += hist[(((size_t)s * copies + c) * passes + pass) * R + tid];
      const uint32_t ex = block_scan(h, sm.scan, &total);
      if (tid < R) sm.base[tid] = sg.off + ex;
      if constexpr (MODE == 2) {
        if (lt == 0 && tid < R) {
          msd.bstart[(size_t)s * R + tid] = sg.off + ex;
          if (h > kWaveCap) atomicOr(&msd.plan->big, 1u);
        }
      }
      if constexpr (MODE == 1) {
        // the segments of the second pass: one per value of digit dh
        const uint32_t nt = tid < R ? (h + kTile - 1) / kTile : 0u;
        uint32_t ttot;
        const uint32_t tex = block_scan(nt, sm.scan, &ttot);
        if (tile == 0) {
          if (tid < R) msd.segs2[tid] = SortSeg{sg.off + ex, h, tex, nt};
          if (tid == 0) {
            *msd.hdr2 = SortHdr{R, ttot, total, 0u};
            *msd.plan = MsdPlan{dh, dl, total, 0u};
          }
        }
      }
      cur = s;
    }

    // ---- per digit: wave offsets, tile count, publication, then each
    // wave's first tile position of the digit
    uint32_t count = 0;
    uint32_t wpre[kSortWaves];
    if (tid < R) {
      const uint32_t d = tid;
      uint32_t c = 0;
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        wpre[w] = c;
        c += sm.wave_hist[w][d];
      }
      count = c;
      store_status(&status[(size_t)tile * R + d], (lt == 0 ? kStatusPrefix : kStatusAggregate) | c);
    }
    uint32_t total;
    const uint32_t local = block_scan(count, sm.scan, &total);
    if (tid < R) {
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) sm.wave_hist[w][tid] = local + wpre[w];
    }

    // ---- look-back for the global offsets
    if (tid < R) {
      const uint32_t d = tid;
      const uint32_t gbase = sg.tile_off / kGroup + s;  // group words of this segment
      const bool last_of_group = (lt % kGroup) == kGroup - 1;
      uint32_t prefix = 0;
      uint32_t* gword = last_of_group ? &gstatus[(size_t)(gbase + lt / kGroup) * R + d] : nullptr;
      if (lt > 0) {
        prefix = look_back<K, kTile>(status, gstatus, keys_in, sg, gbase, lt, R, shift, d, count, gword,
                                     counted ? kFallbackSpinsCounted : kFallbackSpins);
        store_status(&status[(size_t)tile * R + d], kStatusPrefix | (prefix + count));
      }
      if (gword) store_status(gword, kStatusPrefix | (prefix + count));
      sm.delta[d] = sm.base[d] + prefix - local;  // modulo 2^32; the sum below is in range
    }
    __syncthreads();

    // ---- reorder the tile in LDS by digit
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const uint32_t pos = wave * (KPT * kWave) + j * kWave + lane;
      if (pos < tile_n) {
        const uint32_t d = (uint32_t)(k[j] >> shift) & (R - 1);
        const uint32_t at = sm.wave_hist[wave][d] + rank[j];
        if (at < kTile) {
          sm.keys[at] = k[j];
          sm.idx[at] = v[j];
        }
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < kSortWaves * R; i += kSortThreads) (&sm.wave_hist[0][0])[i] = 0;

    // ---- prefetch the next tile, then write this one's digit runs
    const uint32_t seg_end = sg.off + sg.n;
    const uint32_t next = counted ? sm.ticket : tile + gridDim.x;
    const uint32_t s_next = next < T && nseg != 1 ? seg_of_tile(segs, nseg, next) : s;
    const SortSeg sg_next = next < T && nseg != 1 ? segs[s_next] : sg;
    if (next < T) {
      const uint32_t lt_next = next - sg_next.tile_off;
      load_tile(sg_next.off + lt_next * kTile, min(kTile, sg_next.n - lt_next * kTile));
    }
    for (uint32_t p = tid; p < tile_n; p += kSortThreads) {
      const K key = sm.keys[p];
      const uint32_t d = (uint32_t)(key >> shift) & (R - 1);
      const uint32_t out = sm.delta[d] + p;
      if (out < seg_end) {  // always true when the histograms are consistent
        const uint32_t v = sm.idx[p];
        if (keys_out) keys_out[out] = key;
        idx_out[out] = v;
        if (gather_out) {
          // the gather fused into the last pass: the record of ray v moves to
          // its sorted slot (an index outside the rays yields a NaN record)
          const float nan = __int_as_float(0x7fc00000);
          float4 a = make_float4(nan, nan, nan, nan), b = a;
          if (v < gather_n) {
            a = gather_in[2 * (size_t)v];
            b = gather_in[2 * (size_t)v + 1];
          }
          gather_out[2 * (size_t)out] = a;
          gather_out[2 * (size_t)out + 1] = b;
        }
      }
    }
    tile = next;
    s = s_next;
    sg = sg_next;
  }
}

// ---------------------------------------------------------------------------
// The last kernel of the most-significant-digit sort.  After its two scatter
// passes the keys are grouped into buckets of equal (dh, dl) digits, in
// bucket order, each bucket in input order.  Block b takes the buckets that
// start in its window of kLocWindow positions and collects consecutive ones
// into batches of at most kLocCap keys (where a batch ends is found from the
// keys themselves: a bucket starts where the bucket number changes, and its
// size is known).  A batch is sorted in LDS by stable counting passes over
// the other digits in which its keys differ, least significant first, and
// then over the bucket number relative to the batch's first bucket, which
// restores the bucket order.  A bucket larger than a batch is sorted by its
// block alone with the same stable passes run chunk by chunk through global
// memory, the alternate buffers taking every other pass.
constexpr int kLocThreads = 1024;
constexpr int kLocWaves = kLocThreads / kWave;
constexpr int kLocKpt = 8;
constexpr uint32_t kLocCap = kLocThreads * kLocKpt;  // keys of a batch
constexpr uint32_t kLocWindow = kLocCap;             // positions whose buckets a block takes

template <typename K>
struct LocSmem {
  K keys[kLocCap];
  uint32_t idx[kLocCap];
  // per-wave digit counts, then each wave's exclusive prefix per digit; two
  // buffers used in turn, each cleared while the other one is in use
  uint32_t wave_hist[2][kLocWaves][256];
  uint32_t base[256];           // exclusive digit offsets of the last ranking
  uint32_t cnt[256];            // digit counts of the last ranking
  uint32_t run[256];            // large bucket: next output position per digit
  uint32_t fh[sizeof(K)][256];  // large bucket: its digit histograms
  uint32_t scan[kLocWaves];
  uint32_t red[4];
};

// Exclusive scan of one value per thread over a block of NW waves.
template <int NW>
__device__ __forceinline__ uint32_t block_scan_n(uint32_t v, uint32_t* s, uint32_t* total) {
  const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == kWave - 1) s[wave] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t t = s[w];
    pre += (uint32_t)w < wave ? t : 0u;
    tot += t;
  }
  *total = tot;
  __syncthreads();
  return pre + x - v;
}

// Exclusive scan over the 64 lanes of a wave; *total receives the sum.
__device__ __forceinline__ uint32_t wave_scan_excl(uint32_t v, uint32_t* total) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= (uint32_t)off) x += y;
  }
  *total = __shfl(x, kWave - 1, kWave);
  return x - v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v = max(v, (uint32_t)__shfl_xor(v, off, kWave));
  return v;
}

// Position of element j of this thread in a batch: waves own kLocKpt
// consecutive groups of 64.
__device__ __forceinline__ uint32_t loc_pos(int j) {
  return ((threadIdx.x / kWave) * kLocKpt + (uint32_t)j) * kWave + (threadIdx.x & (kWave - 1));
}

// Stable ranking by the 8-bit digits dg of the batch positions below nb,
// with counter buffer buf (zero on entry): pos[j] receives the place of
// element j in the order by digit that keeps equal digits in position
// order.  Leaves the digit counts in sm.cnt and their exclusive offsets in
// sm.base.  The caller synchronises the block after its last use of pos
// and then clears buffer buf (loc_clear) before that buffer's next ranking.
template <typename K>
__device__ void loc_rank(LocSmem<K>& sm, uint32_t buf, const uint32_t (&dg)[kLocKpt], uint32_t nb,
                         uint32_t (&pos)[kLocKpt]) {
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  uint32_t (*wh)[256] = sm.wave_hist[buf];
  uint32_t rank[kLocKpt], old[kLocKpt];
#pragma unroll
  for (int j = 0; j < kLocKpt; ++j) {
    const bool ok = loc_pos(j) < nb;
    const uint64_t peers = match_digit<8>(dg[j], __ballot(ok));
    const uint32_t leader = ok ? (uint32_t)__builtin_ctzll(peers) : lane;
    rank[j] = lanes_below(peers) | (leader << 16);
    old[j] = 0;
    if (ok && lane == leader) old[j] = atomicAdd(&wh[wave][dg[j]], (uint32_t)__popcll(peers));
  }
#pragma unroll
  for (int j = 0; j < kLocKpt; ++j) rank[j] = (rank[j] & 0xFFFFu) + __shfl(old[j], (int)(rank[j] >> 16), kWave);
  __syncthreads();
  if (wave == 0) {
    // lane l takes digits l, l + 64, l + 128, l + 192: each wave's count
    // becomes its exclusive prefix over the waves, then the digit totals
    // are scanned in digit order
#pragma unroll 1
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t d = lane + 64u * q;
      uint32_t t[kLocWaves];
#pragma unroll
      for (int w = 0; w < kLocWaves; ++w) t[w] = wh[w][d];
      uint32_t acc = 0;
#pragma unroll
      for (int w = 0; w < kLocWaves; ++w) {
        wh[w][d] = acc;
        acc += t[w];
      }
      sm.cnt[d] = acc;
    }
    uint32_t c[4], e[4], g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = sm.cnt[lane + 64u * (uint32_t)q];
#pragma unroll
    for (int q = 0; q < 4; ++q) e[q] = wave_scan_excl(c[q], &g[q]);
    uint32_t b = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sm.base[lane + 64u * (uint32_t)q] = b + e[q];
      b += g[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kLocKpt; ++j)
    if (loc_pos(j) < nb) pos[j] = sm.base[dg[j]] + wh[wave][dg[j]] + rank[j];
}

// Clears counter buffer buf (after a block synchronisation that follows its
// last use).
template <typename K>
__device__ __forceinline__ void loc_clear(LocSmem<K>& sm, uint32_t buf) {
  for (uint32_t i = threadIdx.x; i < kLocWaves * 256; i += kLocThreads) (&sm.wave_hist[buf][0][0])[i] = 0;
}

// One stable pass of a batch in LDS: the elements held in registers move to
// their places in the order by dg, and each thread then holds the elements
// of its positions again.  Uses counter buffer buf, which it clears, and
// flips buf for the next pass.
template <typename K>
__device__ void loc_pass(LocSmem<K>& sm, uint32_t& buf, K (&k)[kLocKpt], uint32_t (&v)[kLocKpt],
                         const uint32_t (&dg)[kLocKpt], uint32_t nb) {
  uint32_t pos[kLocKpt];
  loc_rank(sm, buf, dg, nb, pos);
#pragma unroll
  for (int j = 0; j < kLocKpt; ++j) {
    if (loc_pos(j) < nb) {
      sm.keys[pos[j]] = k[j];
      sm.idx[pos[j]] = v[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kLocKpt; ++j) {
    const uint32_t p = loc_pos(j);
    if (p < nb) {
      k[j] = sm.keys[p];
      v[j] = sm.idx[p];
    }
  }
  loc_clear(sm, buf);
  buf ^= 1u;
  // the next pass writes sm.keys only after the synchronisation inside its
  // ranking, when every thread has read its elements back
}

// The ray gather of the fused call for sorted positions [i0, i1).
__device__ __forceinline__ void loc_gather_one(const float4* __restrict__ in, float4* __restrict__ out, uint32_t n_in,
                                               uint32_t at, uint32_t v) {
  const float nan = __int_as_float(0x7fc00000);
  float4 a = make_float4(nan, nan, nan, nan), b = a;
  if (v < n_in) {
    a = in[2 * (size_t)v];
    b = in[2 * (size_t)v + 1];
  }
  out[2 * (size_t)at] = a;
  out[2 * (size_t)at + 1] = b;
}

// A bucket of m > kLocCap keys at [r0, r0 + m), sorted by this block alone:
// the histograms of its digits (all but dh and dl, which its keys share),
// then one stable pass per digit that differs, least significant first,
// chunk by chunk in position order, between the buffers and the alternate
// buffers at the same positions.
template <typename K>
__device__ void loc_big(LocSmem<K>& sm, uint32_t& buf, K* __restrict__ keys, uint32_t* __restrict__ idx,
                        K* __restrict__ kalt, uint32_t* __restrict__ ialt, uint32_t r0, uint32_t m, uint32_t dh,
                        uint32_t dl, const float4* __restrict__ gather_in, float4* __restrict__ gather_out,
                        uint32_t gather_n) {
  constexpr uint32_t P = sizeof(K);
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < P * 256; i += kLocThreads) (&sm.fh[0][0])[i] = 0;
  __syncthreads();
  const K kfirst = keys[r0];
  for (uint32_t i = r0 + tid; i < r0 + m; i += kLocThreads) {
    const K x = keys[i];
    for (uint32_t d = 0; d < P; ++d)
      if (d != dh && d != dl) atomicAdd(&sm.fh[d][(uint32_t)(x >> (8 * d)) & 255u], 1u);
  }
  __syncthreads();
  K* sk = keys;
  uint32_t* si = idx;
  K* dk = kalt;
  uint32_t* di = ialt;
#pragma unroll 1
  for (uint32_t d = 0; d < P; ++d) {
    if (d == dh || d == dl) continue;
    if (sm.fh[d][(uint32_t)(kfirst >> (8 * d)) & 255u] == m) continue;  // the same in every key
    uint32_t tot;
    const uint32_t ex = block_scan_n<kLocWaves>(tid < 256 ? sm.fh[d][tid] : 0u, sm.scan, &tot);
    if (tid < 256) sm.run[tid] = r0 + ex;
    __syncthreads();
    for (uint32_t c0 = r0; c0 < r0 + m; c0 += kLocCap) {
      const uint32_t nb = min(kLocCap, r0 + m - c0);
      K k[kLocKpt];
      uint32_t v[kLocKpt], dg[kLocKpt], pos[kLocKpt];
#pragma unroll
      for (int j = 0; j < kLocKpt; ++j) {
        const uint32_t p = loc_pos(j);
        k[j] = p < nb ? sk[c0 + p] : (K)0;
        v[j] = p < nb ? si[c0 + p] : 0u;
        dg[j] = (uint32_t)(k[j] >> (8 * d)) & 255u;
      }
      loc_rank(sm, buf, dg, nb, pos);
#pragma unroll
      for (int j = 0; j < kLocKpt; ++j) {
        if (loc_pos(j) < nb) {
          const uint32_t out = sm.run[dg[j]] + (pos[j] - sm.base[dg[j]]);
          dk[out] = k[j];
          di[out] = v[j];
        }
      }
      __syncthreads();
      loc_clear(sm, buf);
      buf ^= 1u;
      if (tid < 256) sm.run[tid] += sm.cnt[tid];
      __syncthreads();
    }
    K* tk = sk; sk = dk; dk = tk;
    uint32_t* ti = si; si = di; di = ti;
  }
  if (sk != keys) {
    for (uint32_t i = r0 + tid; i < r0 + m; i += kLocThreads) {
      if (!gather_out) keys[i] = sk[i];
      idx[i] = si[i];
    }
  }
  __syncthreads();
  if (gather_out)
    for (uint32_t i = r0 + tid; i < r0 + m; i += kLocThreads) loc_gather_one(gather_in, gather_out, gather_n, i, idx[i]);
  __syncthreads();
}

template <typename K>
__global__ __launch_bounds__(kLocThreads) void k_msd_local(K* __restrict__ keys, uint32_t* __restrict__ idx,
                                                           K* __restrict__ kalt, uint32_t* __restrict__ ialt,
                                                           const SortHdr* hdr, const MsdPlan* plan,
                                                           const uint32_t* __restrict__ bstart,
                                                           const uint32_t* __restrict__ bcount,
                                                           const float4* __restrict__ gather_in,
                                                           float4* __restrict__ gather_out, uint32_t gather_n) {
  __shared__ LocSmem<K> sm;
  constexpr uint32_t P = sizeof(K);
  const uint32_t n = hdr->total_keys;
  const uint32_t wb = blockIdx.x * kLocWindow;
  if (wb >= n || !plan->big) return;  // k_msd_wave has sorted every bucket
  const uint32_t we = min(n, wb + kLocWindow);
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1);
  for (uint32_t i = tid; i < 2 * kLocWaves * 256; i += kLocThreads) (&sm.wave_hist[0][0][0])[i] = 0;
  __syncthreads();
  uint32_t buf = 0;  // counter buffer of the next ranking
  const uint32_t dh = plan->dh, dl = plan->dl;
  const uint32_t sh = dh * 8, sl = dl * 8;
  auto bucket = [&](K x) -> uint32_t { return (((uint32_t)(x >> sh) & 255u) << 8) | ((uint32_t)(x >> sl) & 255u); };
  // the first bucket that starts in the window
  uint32_t p0;
  {
    const uint32_t j = bucket(keys[wb]);
    const uint32_t st = bstart[j];
    p0 = st == wb ? wb : st + bcount[j];
  }
  while (p0 < we) {  // block-uniform
    const uint32_t lim = min(kLocCap, n - p0);
    K k[kLocKpt];
    uint32_t v[kLocKpt];
#pragma unroll
    for (int j = 0; j < kLocKpt; ++j) {
      const uint32_t p = loc_pos(j);
      k[j] = p < lim ? keys[p0 + p] : (K)0;
      v[j] = p < lim ? idx[p0 + p] : 0u;
    }
    if (tid < 4) sm.red[tid] = 0;
#pragma unroll
    for (int j = 0; j < kLocKpt; ++j) {
      const uint32_t p = loc_pos(j);
      if (p < lim) sm.keys[p] = k[j];
    }
    __syncthreads();
    const K kfirst = sm.keys[0];
    const uint32_t b0 = bucket(kfirst);
    // the batch ends at the end of the last bucket that starts in the window
    // and ends within kLocCap keys of p0
    uint32_t cand = 0;
#pragma unroll
    for (int j = 0; j < kLocKpt; ++j) {
      const uint32_t p = loc_pos(j);
      if (p < lim && p0 + p < we) {
        const uint32_t bj = bucket(k[j]);
        if (p == 0 || bucket(sm.keys[p - 1]) != bj) {
          const uint32_t e = p + bcount[bj];
          if (e <= lim && e > cand) cand = e;
        }
      }
    }
    cand = wave_max(cand);
    if (lane == 0 && cand) atomicMax(&sm.red[0], cand);
    __syncthreads();
    const uint32_t nb = sm.red[0];
    if (nb == 0) {
      // the bucket at p0 does not fit a batch (its size is bounded by the
      // keys that remain, so that every access stays in range)
      const uint32_t m = max(1u, min(bcount[b0], n - p0));
      __syncthreads();
      loc_big(sm, buf, keys, idx, kalt, ialt, p0, m, dh, dl, gather_in, gather_out, gather_n);
      p0 += m;
      continue;
    }
    // digits in which the batch's keys differ (one bit per digit, one LDS
    // atomic per wave), and its bucket span: bucket numbers ascend with the
    // position, so the last element's bucket gives it
    uint64_t diff = 0;
#pragma unroll
    for (int j = 0; j < kLocKpt; ++j) {
      const uint32_t p = loc_pos(j);
      if (p < nb) diff |= (uint64_t)(k[j] ^ kfirst);
      if (p + 1 == nb) sm.red[3] = bucket(k[j]) - b0;
    }
    uint32_t dmask = 0;
#pragma unroll
    for (uint32_t d = 0; d < P; ++d)
      if (__ballot(((diff >> (8 * d)) & 255u) != 0)) dmask |= 1u << d;
    if (lane == 0 && dmask) atomicOr(&sm.red[1], dmask);
    __syncthreads();
    const uint32_t dm = sm.red[1];
    const uint32_t span = sm.red[3];
    bool moved = false;
    uint32_t dg[kLocKpt];
#pragma unroll 1
    for (uint32_t d = 0; d < P; ++d) {
      if (d == dh || d == dl || ((dm >> d) & 1u) == 0) continue;
#pragma unroll
      for (int j = 0; j < kLocKpt; ++j) dg[j] = (uint32_t)(k[j] >> (8 * d)) & 255u;
      loc_pass(sm, buf, k, v, dg, nb);
      moved = true;
    }
    // keys equal in every other digit are still in bucket order
    if (moved && span > 0) {
#pragma unroll 1
      for (uint32_t q = 0; q < (span > 255 ? 16u : 8u); q += 8) {
#pragma unroll
        for (int j = 0; j < kLocKpt; ++j) dg[j] = ((bucket(k[j]) - b0) >> q) & 255u;
        loc_pass(sm, buf, k, v, dg, nb);
      }
    }
#pragma unroll
    for (int j = 0; j < kLocKpt; ++j) {
      const uint32_t p = loc_pos(j);
      if (p < nb) {
        if (moved) {
          if (!gather_out) keys[p0 + p] = k[j];
          idx[p0 + p] = v[j];
        }
        if (gather_out) loc_gather_one(gather_in, gather_out, gather_n, p0 + p, v[j]);
      }
    }
    p0 += nb;
    __syncthreads();  // sm.keys and sm.red are reused by the next batch
  }
}

// The last kernel of the most-significant-digit sort when every (dh, dl)
// bucket holds at most kWaveCap keys (random keys up to ~16M pairs): wave w
// sorts bucket w alone (a bucket's passes are a chain of dependent LDS
// operations, so every bucket gets a wave of its own), the keys in
// registers (kWaveKpt per lane, position lane + 64 j), by stable counting
// passes over the digits other than dh and dl in which the
// bucket's keys differ, least significant first.  A pass ranks the keys
// row by row with wave64 ballots (the lowest lane of each group of equal
// digits adds the group's size to the wave's counter with one LDS atomic),
// scans the 256 counters across the wave and moves the keys through the
// wave's own LDS.  One wave's LDS operations take effect in order, so no
// block barrier is needed; a wave barrier (no instruction) at each
// exchange between lanes keeps the compiler from moving LDS accesses
// across it.  A bucket sits at [bstart, bstart + bcount) after the
// dl pass and the keys there are in input order, so the result is the
// stable sort.  The gather of the fused call moves each ray to its slot.
constexpr int kWaveThreads = 256;
constexpr int kWaveWaves = kWaveThreads / kWave;
constexpr int kWaveKpt = kWaveCap / kWave;
constexpr uint32_t kBuckets = 1u << 16;
constexpr uint32_t kWaveGrid = kBuckets / kWaveWaves;  // one wave per bucket

template <typename K>
struct WaveSmem {
  K keys[kWaveWaves][kWaveCap];
  uint32_t idx[kWaveWaves][kWaveCap];
  uint32_t cnt[kWaveWaves][256];
};

template <typename K>
__global__ __launch_bounds__(kWaveThreads) void k_msd_wave(K* __restrict__ keys, uint32_t* __restrict__ idx,
                                                           const MsdPlan* plan, const uint32_t* __restrict__ bstart,
                                                           const uint32_t* __restrict__ bcount,
                                                           const float4* __restrict__ gather_in,
                                                           float4* __restrict__ gather_out, uint32_t gather_n) {
  if (plan->big) return;  // k_msd_local sorts every bucket
  __shared__ WaveSmem<K> sm;
  constexpr uint32_t P = sizeof(K);
  const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  K* const lk = sm.keys[wv];
  uint32_t* const li = sm.idx[wv];
  uint32_t* const lc = sm.cnt[wv];
  const uint32_t b = blockIdx.x * kWaveWaves + wv;  // this wave's bucket
  const uint32_t dh = plan->dh, dl = plan->dl;
  const uint32_t m = b < kBuckets ? bcount[b] : 0u;
  if (m == 0) return;
  const uint32_t p0 = bstart[b];
  const uint32_t rows = (m + kWave - 1) / kWave;  // rows of keys in use
  K k[kWaveKpt];
  uint32_t v[kWaveKpt];
#pragma unroll
  for (int j = 0; j < kWaveKpt; ++j) {
    const uint32_t p = lane + kWave * j;
    k[j] = p < m ? keys[p0 + p] : (K)0;
    v[j] = p < m ? idx[p0 + p] : 0u;
  }
  bool moved = false;
  if (m > 1) {
    // digits in which the bucket's keys differ
    const K kf = (K)__shfl((unsigned long long)k[0], 0, kWave);
    uint64_t diff = 0;
#pragma unroll
    for (int j = 0; j < kWaveKpt; ++j)
      if (lane + kWave * j < m) diff |= (uint64_t)(k[j] ^ kf);
    uint32_t dm = 0;
#pragma unroll
    for (uint32_t d = 0; d < P; ++d)
      if (__ballot(((diff >> (8 * d)) & 255u) != 0)) dm |= 1u << d;
#pragma unroll 1
    for (uint32_t d = 0; d < P; ++d) {
      if (d == dh || d == dl || ((dm >> d) & 1u) == 0) continue;
      moved = true;
      __builtin_amdgcn_wave_barrier();  // the last pass's reads of lc, lk and li are done
      for (uint32_t i = lane; i < 256; i += kWave) lc[i] = 0;
      __builtin_amdgcn_wave_barrier();
      uint32_t dg[kWaveKpt], rank[kWaveKpt], old[kWaveKpt];
#pragma unroll
      for (int j = 0; j < kWaveKpt; ++j) {
        dg[j] = 0;
        rank[j] = 0;
        old[j] = 0;
        if ((uint32_t)j < rows) {  // wave-uniform
          const uint32_t p = lane + kWave * j;
          const bool ok = p < m;
          dg[j] = (uint32_t)(k[j] >> (8 * d)) & 255u;
          const uint64_t peers = match_digit<8>(dg[j], __ballot(ok));
          const uint32_t leader = ok ? (uint32_t)__builtin_ctzll(peers) : lane;
          rank[j] = lanes_below(peers) | (leader << 16);
          if (ok && lane == leader) old[j] = atomicAdd(&lc[dg[j]], (uint32_t)__popcll(peers));
        }
      }
#pragma unroll
      for (int j = 0; j < kWaveKpt; ++j)
        if ((uint32_t)j < rows)
          rank[j] = (rank[j] & 0xFFFFu) + (uint32_t)__shfl((int)old[j], (int)(rank[j] >> 16), kWave);
      __builtin_amdgcn_wave_barrier();
      // exclusive offsets of the 256 digits: lane l owns digits 4l .. 4l + 3
      const uint32_t c0 = lc[4 * lane], c1 = lc[4 * lane + 1], c2 = lc[4 * lane + 2], c3 = lc[4 * lane + 3];
      uint32_t tot;
      const uint32_t ex = wave_scan_excl(c0 + c1 + c2 + c3, &tot);
      lc[4 * lane] = ex;
      lc[4 * lane + 1] = ex + c0;
      lc[4 * lane + 2] = ex + c0 + c1;
      lc[4 * lane + 3] = ex + c0 + c1 + c2;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < kWaveKpt; ++j) {
        if (lane + kWave * j < m) {
          const uint32_t at = lc[dg[j]] + rank[j];
          lk[at] = k[j];
          li[at] = v[j];
        }
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < kWaveKpt; ++j) {
        const uint32_t p = lane + kWave * j;
        if (p < m) {
          k[j] = lk[p];
          v[j] = li[p];
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kWaveKpt; ++j) {
    const uint32_t p = lane + kWave * j;
    if (p < m) {
      if (moved) {
        if (!gather_out) keys[p0 + p] = k[j];
        idx[p0 + p] = v[j];
      }
      if (gather_out) loc_gather_one(gather_in, gather_out, gather_n, p0 + p, v[j]);
    }
  }
}

template <typename F>
uint32_t resident(F kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per <= 0) per = 1;
  return (uint32_t)(cus * per);
}

template <typename K, int DB, int KPT>
struct Resident {
  static uint32_t hist() {
    static const uint32_t v = resident(k_seg_hist<K, DB, KPT>, kSortThreads);
    return v;
  }
  template <int MODE = 0>
  static uint32_t pass() {
    static const uint32_t v = resident(k_seg_pass<K, DB, KPT, MODE>, kSortThreads);
    return v;
  }
};

template <int KIND, typename K>
uint32_t keys_hist_resident() {
  static const uint32_t v = resident(k_keys_hist<KIND, K>, kSortThreads);
  return v;
}

// Launches k_keys_hist for the key family of P (8-bit digits).
template <typename K>
void launch_keys_hist(const KeyPlan& P, uint32_t units, const float4* rays, uint32_t n, K* keys, uint32_t* idx,
                      uint32_t passes, uint32_t copies, uint32_t* hist, uint32_t* status, uint32_t status_stride,
                      uint32_t tiles, uint32_t* gstatus, uint32_t gstatus_stride, uint32_t groups,
                      uint32_t clear_passes, hipStream_t st) {
#define RR_KEYS_HIST(F)                                                                                           \
  hipLaunchKernelGGL((k_keys_hist<F, K>), dim3(std::max(1u, std::min(units, std::min(keys_hist_resident<F, K>(), \
                                                                                       1024u)))),              \
                     dim3(kSortThreads), 0, st, rays, n, P, keys, idx, passes, copies, hist, status, status_stride, \
                     tiles, gstatus, gstatus_stride, groups, clear_passes)
  const int f = key_family(P.kind);
  if (f == 1) RR_KEYS_HIST(1);
  else if (f == 2) RR_KEYS_HIST(2);
  else if constexpr (sizeof(K) == 4) RR_KEYS_HIST(3);
#undef RR_KEYS_HIST
}

// A dense single-segment sort whose keys k_keys_hist computes from rays.
struct KeySource {
  const rr_ray* rays;
  KeyPlan plan;
};

template <typename K, int DB, int KPT>
rr_status seg_sort_impl(K* keys, uint32_t* idx, const SegLayout& L, char* ws, SortHdr* hdr_ext, SortSeg* segs_ext,
                        const uint32_t* count_dev, uint32_t n_max, bool counted, const rr_ray* gather_in,
                        rr_ray* gather_out, uint32_t gather_n, hipStream_t st, const KeySource* ksrc = nullptr) {
  constexpr uint32_t R = 1u << DB;
  K* kalt = reinterpret_cast<K*>(ws + L.keys_alt);
  uint32_t* ialt = reinterpret_cast<uint32_t*>(ws + L.idx_alt);
  const bool single = hdr_ext == nullptr;
  SortHdr* hdr = single ? reinterpret_cast<SortHdr*>(ws + L.hdr) : hdr_ext;
  SortSeg* segs = single ? reinterpret_cast<SortSeg*>(ws + L.segs) : segs_ext;
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  uint32_t* status = reinterpret_cast<uint32_t*>(ws + L.status);
  uint32_t* gstatus = reinterpret_cast<uint32_t*>(ws + L.gstatus);
  uint32_t* counters = reinterpret_cast<uint32_t*>(ws + L.counters);

  const uint32_t hist_res = Resident<K, DB, KPT>::hist();
  const uint32_t pass_res = Resident<K, DB, KPT>::pass();
  const uint32_t max_tiles = L.max_tiles;
  const uint32_t hist_words = L.hist_copies * L.passes * R;  // per segment
  if (single)
    hipLaunchKernelGGL(k_seg_setup_single, dim3(L.hist_copies), dim3(256), 0, st, count_dev, n_max, L.tile, hdr,
                       segs, hist, hist_words, counters, L.passes);
  else
    hipLaunchKernelGGL(k_seg_init, dim3(std::max(1u, std::min(64u, L.max_seg))), dim3(256), 0, st, hdr, hist,
                       hist_words, counters, L.passes);
  // about one unit per block: each block flushes its whole histogram with
  // global atomics, so more blocks than units only adds flush traffic
  if (ksrc) {
    // keys from the rays, counted in the same kernel (n_max keys, no device count)
    const uint32_t tiles = (n_max + L.tile - 1) / L.tile;
    if constexpr (DB == 8)
      launch_keys_hist<K>(ksrc->plan, (n_max + kHistUnit - 1) / kHistUnit,
                          reinterpret_cast<const float4*>(ksrc->rays), n_max, keys, idx, L.passes, L.hist_copies, hist,
                          status, L.status_stride, tiles, gstatus, L.gstatus_stride, tiles / kGroup + 1, L.passes, st);
  } else {
    const uint32_t hist_units = std::max(1u, max_tiles * L.tile / kHistUnit);
    const uint32_t hist_blocks = std::max(1u, std::min(hist_units, std::min(hist_res, 1024u)));
    hipLaunchKernelGGL((k_seg_hist<K, DB, KPT>), dim3(hist_blocks), dim3(kSortThreads), 0, st, keys, hdr, segs,
                       L.passes, L.hist_copies, hist, status, L.status_stride, gstatus, L.gstatus_stride,
                       (const MsdPlan*)nullptr, L.passes, 0u, 0u);
  }
  // one resident wave of blocks
  const uint32_t pass_blocks = std::max(1u, std::min(max_tiles, pass_res));
  K* src_k = keys;
  uint32_t* src_i = idx;
  K* dst_k = kalt;
  uint32_t* dst_i = ialt;
  for (uint32_t p = 0; p < L.passes; ++p) {
    // the last pass of a sort with a fused gather writes the rays instead of the keys
    const bool g = gather_out && p + 1 == L.passes;
    hipLaunchKernelGGL((k_seg_pass<K, DB, KPT>), dim3(pass_blocks), dim3(kSortThreads), 0, st, src_k, src_i,
                       g ? nullptr : dst_k, dst_i, hdr, segs, p * DB, L.passes, p, L.hist_copies, hist,
                       status + (size_t)p * L.status_stride, gstatus + (size_t)p * L.gstatus_stride,
                       counted ? counters + p : nullptr, g ? reinterpret_cast<const float4*>(gather_in) : nullptr,
                       g ? reinterpret_cast<float4*>(gather_out) : nullptr, gather_n, MsdArgs{});
    std::swap(src_k, dst_k);
    std::swap(src_i, dst_i);
  }
  RR_LAUNCH_CHECK();
  // an even pass count leaves the result in the caller's buffers
  return RR_OK;
}

template <typename K>
uint32_t msd_local_blocks(uint32_t n_max) {
  return std::max(1u, (n_max + kLocWindow - 1) / kLocWindow);
}

// The most-significant-digit sort of one segment of min(*count_dev, n_max)
// keys (n_max with keys from the rays): histograms of every digit, a stable
// pass on the highest differing digit dh, histograms of the next one (dl)
// per dh value, a stable pass on dl within each dh value, then each (dh, dl)
// bucket sorted on its remaining digits by k_msd_local.  Every step keeps
// equal keys in input order, so the result is the stable sort.
template <typename K, int KPT>
rr_status msd_sort_impl(K* keys, uint32_t* idx, const SegLayout& L, char* ws, const uint32_t* count_dev,
                        uint32_t n_max, const rr_ray* gather_in, rr_ray* gather_out, uint32_t gather_n,
                        hipStream_t st, const KeySource* ksrc = nullptr) {
  constexpr uint32_t R = 256;
  K* kalt = reinterpret_cast<K*>(ws + L.keys_alt);
  uint32_t* ialt = reinterpret_cast<uint32_t*>(ws + L.idx_alt);
  SortHdr* hdr = reinterpret_cast<SortHdr*>(ws + L.hdr);
  SortSeg* segs = reinterpret_cast<SortSeg*>(ws + L.segs);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  MsdPlan* plan = reinterpret_cast<MsdPlan*>(ws + L.plan);
  SortHdr* hdr2 = reinterpret_cast<SortHdr*>(ws + L.hdr2);
  SortSeg* segs2 = reinterpret_cast<SortSeg*>(ws + L.segs2);
  uint32_t* hist2 = reinterpret_cast<uint32_t*>(ws + L.hist2);
  uint32_t* bstart = reinterpret_cast<uint32_t*>(ws + L.bstart);
  uint32_t* status2 = reinterpret_cast<uint32_t*>(ws + L.status2);
  uint32_t* gstatus2 = reinterpret_cast<uint32_t*>(ws + L.gstatus2);

  const uint32_t hist_res = Resident<K, 8, KPT>::hist();
  const uint32_t hist_words = L.hist_copies * L.passes * R;
  hipLaunchKernelGGL(k_msd_setup, dim3(64), dim3(256), 0, st, count_dev, n_max, L.tile, hdr, segs, hist, hist_words,
                     hist2, R * R, hdr2, plan);
  // histograms of every digit; the look-back words of both passes are
  // cleared for up to R more tiles (the second pass's segments each add a
  // partial tile) and their groups
  const uint32_t tiles = (n_max + L.tile - 1) / L.tile;
  if (ksrc) {
    launch_keys_hist<K>(ksrc->plan, (n_max + kHistUnit - 1) / kHistUnit, reinterpret_cast<const float4*>(ksrc->rays),
                        n_max, keys, idx, L.passes, L.hist_copies, hist, status2, L.status2_stride, tiles + R,
                        gstatus2, L.gstatus2_stride, (tiles + R) / kGroup + R + 2, 2u, st);
  } else {
    const uint32_t units = std::max(1u, tiles * L.tile / kHistUnit);
    hipLaunchKernelGGL((k_seg_hist<K, 8, KPT>), dim3(std::max(1u, std::min(units, std::min(hist_res, 1024u)))),
                       dim3(kSortThreads), 0, st, keys, hdr, segs, L.passes, L.hist_copies, hist, status2,
                       L.status2_stride, gstatus2, L.gstatus2_stride, (const MsdPlan*)nullptr, 2u, R, R + 1);
  }
  // first pass: by dh, into the alternate buffers
  hipLaunchKernelGGL((k_seg_pass<K, 8, KPT, 1>),
                     dim3(std::max(1u, std::min(L.max_tiles, Resident<K, 8, KPT>::template pass<1>()))),
                     dim3(kSortThreads), 0, st, keys, idx, kalt, ialt, hdr, segs, 0u, L.passes, 0u, L.hist_copies, hist,
                     status2, gstatus2, (uint32_t*)nullptr, (const float4*)nullptr, (float4*)nullptr, 0u,
                     MsdArgs{1u, plan, hdr2, segs2, bstart});
  // digit-dl histograms of every dh segment
  const uint32_t units2 = std::max(1u, (L.max_tiles + R) * L.tile / kHistUnit);
  hipLaunchKernelGGL((k_seg_hist<K, 8, KPT>), dim3(std::max(1u, std::min(units2, std::min(hist_res, 1024u)))),
                     dim3(kSortThreads), 0, st, kalt, hdr2, segs2, 1u, 1u, hist2, (uint32_t*)nullptr, 0u,
                     (uint32_t*)nullptr, 0u, (const MsdPlan*)plan, 0u, 0u, 0u);
  // second pass: by dl within each dh segment, back into the caller's buffers
  hipLaunchKernelGGL((k_seg_pass<K, 8, KPT, 2>),
                     dim3(std::max(1u, std::min(L.max_tiles + R, Resident<K, 8, KPT>::template pass<2>()))),
                     dim3(kSortThreads), 0, st, kalt, ialt, keys, idx, hdr2, segs2, 0u, 1u, 0u, 1u, hist2,
                     status2 + L.status2_stride, gstatus2 + L.gstatus2_stride, (uint32_t*)nullptr,
                     (const float4*)nullptr, (float4*)nullptr, 0u, MsdArgs{2u, plan, nullptr, nullptr, bstart});
  // every (dh, dl) bucket on its remaining digits (and the ray gather)
  hipLaunchKernelGGL((k_msd_wave<K>), dim3(kWaveGrid), dim3(kWaveThreads), 0, st, keys, idx, (const MsdPlan*)plan,
                     bstart, hist2, reinterpret_cast<const float4*>(gather_in), reinterpret_cast<float4*>(gather_out),
                     gather_n);
  hipLaunchKernelGGL((k_msd_local<K>), dim3(msd_local_blocks<K>(n_max)), dim3(kLocThreads), 0, st, keys, idx, kalt,
                     ialt, hdr, plan, bstart, hist2, reinterpret_cast<const float4*>(gather_in),
                     reinterpret_cast<float4*>(gather_out), gather_n);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

}  // namespace

SegLayout msd_layout(int64_t n_max, uint32_t key_bits, uint32_t kpt) {
  SegLayout L{};
  constexpr size_t R = 256;
  const size_t kb = key_bits / 8;
  L.msd = true;
  L.passes = key_bits / 8;
  L.tile = kSortThreads * kpt;
  L.max_seg = 1;
  L.max_tiles = (uint32_t)((n_max + L.tile - 1) / L.tile + 1);
  L.hist_copies = kHistCopies;
  size_t off = 0;
  L.keys_alt = off; off = align_up(off + kb * (size_t)n_max, 256);
  L.idx_alt = off; off = align_up(off + 4 * (size_t)n_max, 256);
  L.hdr = off; off = align_up(off + sizeof(SortHdr), 256);
  L.segs = off; off = align_up(off + sizeof(SortSeg), 256);
  L.hist = off; off = align_up(off + 4 * (size_t)L.hist_copies * L.passes * R, 256);
  L.counters = off; off = align_up(off + 4 * (size_t)L.passes, 256);
  L.plan = off; off = align_up(off + sizeof(MsdPlan), 256);
  L.hdr2 = off; off = align_up(off + sizeof(SortHdr), 256);
  L.segs2 = off; off = align_up(off + sizeof(SortSeg) * R, 256);
  L.hist2 = off; off = align_up(off + 4 * R * R, 256);
  L.bstart = off; off = align_up(off + 4 * R * R, 256);
  // the second pass has at most max_tiles + R - 1 tiles; group words of
  // segment s sit at tile_off / kGroup + s + lt / kGroup
  const size_t tiles2 = (size_t)L.max_tiles + R;
  L.status2_stride = (uint32_t)(tiles2 * R);
  L.status2 = off; off = align_up(off + 4 * 2 * (size_t)L.status2_stride, 256);
  L.gstatus2_stride = (uint32_t)((tiles2 / kGroup + R + 2) * R);
  L.gstatus2 = off; off = align_up(off + 4 * 2 * (size_t)L.gstatus2_stride, 256);
  L.status = L.status2;
  L.gstatus = L.gstatus2;
  L.status_stride = L.status2_stride;
  L.gstatus_stride = L.gstatus2_stride;
  L.total = off;
  return L;
}

// Which of the two sorts is faster depends on the keys.  Evenly spread keys
// from ~2M to ~17M pairs fill every (dh, dl) bucket with at most kWaveCap
// keys, so k_msd_wave sorts the buckets and the MSD sort beats the LSD sort.
// Clustered keys such as ray keys leave large buckets to k_msd_local, whose
// chains of in-LDS passes run on one block per CU, and the LSD sort is then
// as fast or faster.  Hence rr_sort keeps the LSD sort.  From 2^27 pairs on
// even evenly spread keys give buckets of over 2K keys.
bool msd_supported(int64_t n_max, uint32_t key_bits) {
  return key_bits == 64 && n_max > 0 && n_max < (int64_t(1) << 27);
}


SegLayout seg_layout(int64_t n_max, uint32_t max_seg, uint32_t key_bits, uint32_t db, uint32_t kpt) {
  SegLayout L{};
  const size_t kb = key_bits / 8;
  L.passes = (key_bits + db - 1) / db;
  L.tile = kSortThreads * kpt;
  L.max_seg = max_seg;
  // each segment can add one partial tile
  L.max_tiles = (uint32_t)((n_max + L.tile - 1) / L.tile + max_seg);
  const size_t R = (size_t)1 << db;
  L.status_stride = (uint32_t)(L.max_tiles * R);
  size_t off = 0;
  L.keys_alt = off; off = align_up(off + kb * (size_t)n_max, 256);
  L.idx_alt = off; off = align_up(off + 4 * (size_t)n_max, 256);
  L.hdr = off; off = align_up(off + sizeof(SortHdr), 256);
  L.segs = off; off = align_up(off + sizeof(SortSeg) * max_seg, 256);
  L.hist_copies = max_seg == 1 ? kHistCopies : 1u;
  L.hist = off; off = align_up(off + 4 * (size_t)max_seg * L.hist_copies * L.passes * R, 256);
  L.counters = off; off = align_up(off + 4 * (size_t)L.passes, 256);  // tile counter per pass
  L.status = off; off = align_up(off + 4 * (size_t)L.passes * L.status_stride, 256);
  // group words: group g of a segment whose first tile is t0 and index s
  // sits at t0 / kGroup + s + g, below max_tiles / kGroup + max_seg
  L.gstatus_stride = (uint32_t)((L.max_tiles / kGroup + max_seg + 1) * R);
  L.gstatus = off; off = align_up(off + 4 * (size_t)L.passes * L.gstatus_stride, 256);
  L.total = off;
  return L;
}

uint32_t sort_tile_keys(uint32_t kpt) { return kSortThreads * kpt; }

uint32_t sort_default_kpt(int64_t n) { return n >= (int64_t(1) << 24) ? 16u : 8u; }

bool sort_config_supported(uint32_t key_bits, uint32_t digit_bits, uint32_t kpt) {
  return (key_bits == 32 || key_bits == 64) && (digit_bits == 4 || digit_bits == 8) && (kpt == 8 || kpt == 16);
}

size_t sort_workspace_bytes(int64_t n_max, uint32_t key_bits, uint32_t digit_bits, uint32_t kpt) {
  return seg_layout(n_max, 1, key_bits, digit_bits, kpt).total;
}

size_t sort_workspace_bytes_any(int64_t n_max, uint32_t key_bits) {
  size_t m = 0;
  for (uint32_t db : {4u, 8u})
    for (uint32_t kpt : {8u, 16u}) m = std::max(m, sort_workspace_bytes(n_max, key_bits, db, kpt));
  if (msd_supported(n_max, key_bits)) m = std::max(m, msd_layout(n_max, key_bits, sort_default_kpt(n_max)).total);
  return m;
}

void sort_warm(uint32_t key_bits, uint32_t db, uint32_t kpt) {
#define RR_WARM_CASE(KT, DBV, KPTV)                                  \
  if (sizeof(KT) * 8 == key_bits && db == DBV && kpt == KPTV) {      \
    (void)Resident<KT, DBV, KPTV>::hist();                           \
    (void)Resident<KT, DBV, KPTV>::pass();                           \
    if (sizeof(KT) == 8 && DBV == 8) {                               \
      (void)Resident<KT, DBV, KPTV>::template pass<1>();             \
      (void)Resident<KT, DBV, KPTV>::template pass<2>();             \
    }                                                                \
  }
  RR_WARM_CASE(uint32_t, 8, 16)
  RR_WARM_CASE(uint32_t, 8, 8)
  RR_WARM_CASE(uint32_t, 4, 16)
  RR_WARM_CASE(uint32_t, 4, 8)
  RR_WARM_CASE(uint64_t, 8, 16)
  RR_WARM_CASE(uint64_t, 8, 8)
  RR_WARM_CASE(uint64_t, 4, 16)
  RR_WARM_CASE(uint64_t, 4, 8)
#undef RR_WARM_CASE
}

rr_status launch_seg_sort(void* keys, uint32_t* idx, const SegLayout& L, void* ws, SortHdr* hdr, SortSeg* segs,
                          const uint32_t* count_dev, uint32_t n_max, uint32_t key_bits, uint32_t db, uint32_t kpt,
                          bool counted, hipStream_t st, const rr_ray* gather_in, rr_ray* gather_out,
                          uint32_t gather_n) {
  char* w = reinterpret_cast<char*>(ws);
#define RR_SORT_CASE(KT, DBV, KPTV)                                                                        \
  if (sizeof(KT) * 8 == key_bits && db == DBV && kpt == KPTV)                                            \
    return seg_sort_impl<KT, DBV, KPTV>(reinterpret_cast<KT*>(keys), idx, L, w, hdr, segs, count_dev, n_max, counted, \
                                        gather_in, gather_out, gather_n, st);
  RR_SORT_CASE(uint32_t, 8, 16)
  RR_SORT_CASE(uint32_t, 8, 8)
  RR_SORT_CASE(uint32_t, 4, 16)
  RR_SORT_CASE(uint32_t, 4, 8)
  RR_SORT_CASE(uint64_t, 8, 16)
  RR_SORT_CASE(uint64_t, 8, 8)
  RR_SORT_CASE(uint64_t, 4, 16)
  RR_SORT_CASE(uint64_t, 4, 8)
#undef RR_SORT_CASE
  return RR_ERR_UNSUPPORTED;
}

namespace {

// The most-significant-digit sort with kpt keys per thread in its scatter
// passes (keys from the rays when ksrc is given; the ray gather in its last
// kernel when gather_out is given).
rr_status launch_msd(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                     uint32_t kpt, void* ws, size_t ws_bytes, const rr_ray* gather_in, rr_ray* gather_out,
                     uint32_t gather_n, hipStream_t st, const KeySource* ksrc) {
  const SegLayout L = msd_layout(n_max, key_bits, kpt);
  if (ws_bytes < L.total) return RR_ERR_WORKSPACE_TOO_SMALL;
  char* w = reinterpret_cast<char*>(ws);
#define RR_MSD_CASE(KT, KPTV)                                                                                       \
  if (sizeof(KT) * 8 == key_bits && kpt == KPTV)                                                                  \
    return msd_sort_impl<KT, KPTV>(reinterpret_cast<KT*>(keys), idx, L, w, count_dev, (uint32_t)n_max, gather_in, \
                                   gather_out, gather_n, st, ksrc);
  RR_MSD_CASE(uint32_t, 16)
  RR_MSD_CASE(uint32_t, 8)
  RR_MSD_CASE(uint64_t, 16)
  RR_MSD_CASE(uint64_t, 8)
#undef RR_MSD_CASE
  return RR_ERR_UNSUPPORTED;
}

}  // namespace

rr_status launch_sort_auto(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                           void* ws, size_t ws_bytes, hipStream_t st, bool force_msd) {
  if (key_bits != 32 && key_bits != 64) return RR_ERR_UNSUPPORTED;
  if (force_msd && !msd_supported(n_max, key_bits)) return RR_ERR_UNSUPPORTED;
  const uint32_t kpt = sort_default_kpt(n_max);
  if (force_msd)
    return launch_msd(keys, idx, n_max, count_dev, key_bits, kpt, ws, ws_bytes, nullptr, nullptr, 0u, st, nullptr);
  return launch_sort(keys, idx, n_max, count_dev, key_bits, 8, kpt, ws, ws_bytes, st);
}

rr_status launch_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                      uint32_t db, uint32_t kpt, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!sort_config_supported(key_bits, db, kpt)) return RR_ERR_UNSUPPORTED;
  const SegLayout L = seg_layout(n_max, 1, key_bits, db, kpt);
  if (ws_bytes < L.total) return RR_ERR_WORKSPACE_TOO_SMALL;
  return launch_seg_sort(keys, idx, L, ws, nullptr, nullptr, count_dev, (uint32_t)n_max, key_bits, db, kpt, false,
                         st);
}

rr_status launch_keys_sort_gather(const rr_ray* rays, int64_t n, const KeyPlan& plan, void* keys, uint32_t* idx,
                                  uint32_t kpt, void* ws, size_t ws_bytes, rr_ray* rays_out, hipStream_t st,
                                  bool force_msd) {
  const uint32_t key_bits = plan.key64 ? 64u : 32u;
  if (n <= 0) return RR_OK;
  if (!sort_config_supported(key_bits, 8, kpt) || (plan.key64 && key_family(plan.kind) == 3))
    return RR_ERR_UNSUPPORTED;
  if (force_msd && !msd_supported(n, key_bits)) return RR_ERR_UNSUPPORTED;
  const KeySource src{rays, plan};
  if (force_msd)
    return launch_msd(keys, idx, n, nullptr, key_bits, kpt, ws, ws_bytes, rays, rays_out, (uint32_t)n, st, &src);
  const SegLayout L = seg_layout(n, 1, key_bits, 8, kpt);
  if (ws_bytes < L.total) return RR_ERR_WORKSPACE_TOO_SMALL;
  char* w = reinterpret_cast<char*>(ws);
#define RR_KSORT_CASE(KT, KPTV)                                                                              \
  if (sizeof(KT) * 8 == key_bits && kpt == KPTV)                                                           \
    return seg_sort_impl<KT, 8, KPTV>(reinterpret_cast<KT*>(keys), idx, L, w, nullptr, nullptr, nullptr,   \
                                      (uint32_t)n, false, rays, rays_out, (uint32_t)n, st, &src);
  RR_KSORT_CASE(uint32_t, 16)
  RR_KSORT_CASE(uint32_t, 8)
  RR_KSORT_CASE(uint64_t, 16)
  RR_KSORT_CASE(uint64_t, 8)
#undef RR_KSORT_CASE
  return RR_ERR_UNSUPPORTED;
}

rr_status launch_sort_gather(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                             uint32_t db, uint32_t kpt, void* ws, size_t ws_bytes, const rr_ray* rays_in,
                             rr_ray* rays_out, hipStream_t st, bool force_msd) {
  if (!sort_config_supported(key_bits, db, kpt)) return RR_ERR_UNSUPPORTED;
  if (force_msd && (db != 8 || !msd_supported(n_max, key_bits))) return RR_ERR_UNSUPPORTED;
  if (db == 8 && (force_msd))
    return launch_msd(keys, idx, n_max, count_dev, key_bits, kpt, ws, ws_bytes, rays_in, rays_out, (uint32_t)n_max, st,
                      nullptr);
  const SegLayout L = seg_layout(n_max, 1, key_bits, db, kpt);
  if (ws_bytes < L.total) return RR_ERR_WORKSPACE_TOO_SMALL;
  return launch_seg_sort(keys, idx, L, ws, nullptr, nullptr, count_dev, (uint32_t)n_max, key_bits, db, kpt, false,
                         st, rays_in, rays_out, (uint32_t)n_max);
}

}  // namespace rr
