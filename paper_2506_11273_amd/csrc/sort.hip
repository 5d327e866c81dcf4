// Stable LSD radix sort of (key, index) pairs (Section 3.2 sorts key/index
// pairs with a device-wide radix sort).
//
// Design (one histogram pass, then one scatter pass per digit):
//  * k_sort_hist reads every key once and builds the digit histograms of
//    all passes in LDS; k_sort_scan turns them into per-digit bases.
//  * k_sort_pass takes tiles in launch order from an atomic counter, ranks
//    the tile's keys by digit with wave64 ballots (a match over the digit's
//    bits gives each lane its peers; the lowest peer bumps the wave's digit
//    counter in LDS), publishes the tile's digit counts, looks back over the
//    previous tiles' published counts for its global offsets (decoupled
//    look-back, Merrill and Garland 2016), reorders the tile in LDS and
//    writes each digit run contiguously.
// Ranking keeps input order within a digit, so the sort is stable and the
// output is the unique (key, index) lexicographic order for ascending input
// indices.  Look-back waits are bounded: a wait that exceeds its limit sets
// an error word instead of hanging.
#include <algorithm>
#include <utility>

#include "common.hpp"

namespace rr {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr uint32_t kSpinLimit = 1u << 18;

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t read_count(const uint32_t* count_dev, uint32_t n_max) {
  if (!count_dev) return n_max;
  const uint32_t c = *count_dev;
  return c < n_max ? c : n_max;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_scan_256(uint32_t v, uint32_t* s, uint32_t* total) {
  const uint32_t t = threadIdx.x;
  s[t] = v;
  __syncthreads();
#pragma unroll
  for (uint32_t off = 1; off < kSortThreads; off <<= 1) {
    const uint32_t x = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  const uint32_t incl = s[t];
  *total = s[kSortThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_sort_init(uint32_t* __restrict__ hist, uint32_t n_hist, uint32_t* __restrict__ counters,
                            uint32_t n_counters) {
  for (uint32_t i = threadIdx.x; i < n_hist; i += blockDim.x) hist[i] = 0;
  for (uint32_t i = threadIdx.x; i < n_counters; i += blockDim.x) counters[i] = 0;
}

// Digit histograms of every pass, plus clearing of the look-back words the
// passes will use.
template <typename K, int DB>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const K* __restrict__ keys, const uint32_t* count_dev,
                                                            uint32_t n_max, uint32_t passes,
                                                            uint32_t* __restrict__ hist,
                                                            uint32_t* __restrict__ status, uint32_t tile_keys,
                                                            uint32_t status_pass_stride) {
  constexpr uint32_t R = 1u << DB;
  constexpr uint32_t kMaxPasses = (8 * sizeof(K) + DB - 1) / DB;
  __shared__ uint32_t s_h[kMaxPasses * R];
  for (uint32_t i = threadIdx.x; i < passes * R; i += kSortThreads) s_h[i] = 0;
  __syncthreads();
  const uint32_t n = read_count(count_dev, n_max);
  const uint32_t stride = gridDim.x * kSortThreads;
  for (uint32_t i = blockIdx.x * kSortThreads + threadIdx.x; i < n; i += stride) {
    const K k = keys[i];
    for (uint32_t p = 0; p < passes; ++p) atomicAdd(&s_h[p * R + ((uint32_t)(k >> (p * DB)) & (R - 1))], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < passes * R; i += kSortThreads)
    if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
  // clear the look-back words of the tiles this sort will use
  const uint32_t tiles = (n + tile_keys - 1) / tile_keys;
  const uint32_t words = tiles * R;
  for (uint32_t p = 0; p < passes; ++p)
    for (uint32_t i = blockIdx.x * kSortThreads + threadIdx.x; i < words; i += stride)
      status[(size_t)p * status_pass_stride + i] = 0;
}

// hist[p][d] -> exclusive prefix over d (the first output slot of digit d).
template <int DB>
__global__ __launch_bounds__(kSortThreads) void k_sort_scan(uint32_t* __restrict__ hist, uint32_t passes) {
  constexpr uint32_t R = 1u << DB;
  __shared__ uint32_t s[kSortThreads];
  for (uint32_t p = 0; p < passes; ++p) {
    const uint32_t v = threadIdx.x < R ? hist[p * R + threadIdx.x] : 0u;
    uint32_t total;
    const uint32_t ex = block_scan_256(v, s, &total);
    if (threadIdx.x < R) hist[p * R + threadIdx.x] = ex;
  }
}

template <typename K, int DB, int KPT>
struct PassSmem {
  static constexpr uint32_t R = 1u << DB;
  static constexpr uint32_t kTile = kSortThreads * KPT;
  K keys[kTile];
  uint32_t idx[kTile];
  uint32_t wave_hist[kSortWaves][R];
  uint32_t local_off[R];
  uint32_t global_off[R];
  uint32_t scan[kSortThreads];
  uint32_t tile;
};

template <typename K, int DB, int KPT>
__global__ __launch_bounds__(kSortThreads) void k_sort_pass(const K* __restrict__ keys_in,
                                                            const uint32_t* __restrict__ idx_in,
                                                            K* __restrict__ keys_out, uint32_t* __restrict__ idx_out,
                                                            const uint32_t* count_dev, uint32_t n_max, uint32_t shift,
                                                            const uint32_t* __restrict__ digit_base,
                                                            uint32_t* __restrict__ status, uint32_t* tile_counter,
                                                            uint32_t* err) {
  using S = PassSmem<K, DB, KPT>;
  constexpr uint32_t R = S::R;
  constexpr uint32_t kTile = S::kTile;
  __shared__ S sm;
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;

  if (tid == 0) sm.tile = atomicAdd(tile_counter, 1u);
  for (uint32_t i = tid; i < kSortWaves * R; i += kSortThreads) (&sm.wave_hist[0][0])[i] = 0;
  __syncthreads();
  const uint32_t n = read_count(count_dev, n_max);
  const uint32_t tile = sm.tile;
  const uint32_t tiles = (n + kTile - 1) / kTile;
  if (tile >= tiles) return;  // block-uniform
  const uint32_t base = tile * kTile;
  const uint32_t tile_n = min(kTile, n - base);

  // ---- load (wave-striped: wave w owns KPT consecutive groups of 64)
  K k[KPT];
  uint32_t v[KPT];
  uint32_t rank[KPT];
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const uint32_t pos = wave * (KPT * kWave) + j * kWave + lane;
    const bool ok = pos < tile_n;
    k[j] = ok ? keys_in[base + pos] : (K)0;
    v[j] = ok ? idx_in[base + pos] : 0u;
  }

  // ---- rank within the wave, in (j, lane) order
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const uint32_t pos = wave * (KPT * kWave) + j * kWave + lane;
    const bool ok = pos < tile_n;
    const uint32_t d = (uint32_t)(k[j] >> shift) & (R - 1);
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < DB; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t below = lanes_below(peers);
    const int leader = ok ? (int)__builtin_ctzll(peers) : (int)lane;
    uint32_t old = 0;
    if (ok && (int)lane == leader) {
      old = sm.wave_hist[wave][d];
      sm.wave_hist[wave][d] = old + (uint32_t)__popcll(peers);
    }
    old = __shfl(old, leader, kWave);
    rank[j] = old + below;
  }
  __syncthreads();

  // ---- per digit: wave offsets, tile count, publication
  uint32_t count = 0;
  for (uint32_t d = tid; d < R; d += kSortThreads) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      const uint32_t t = sm.wave_hist[w][d];
      sm.wave_hist[w][d] = c;
      c += t;
    }
    count = c;
    const uint32_t word = (tile == 0 ? kStatusPrefix : kStatusAggregate) | c;
    __hip_atomic_store(&status[(size_t)tile * R + d], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  uint32_t total;
  const uint32_t local = block_scan_256(tid < R ? count : 0u, sm.scan, &total);
  if (tid < R) sm.local_off[tid] = local;

  // ---- decoupled look-back: sum the counts of digit d in earlier tiles
  if (tid < R) {
    const uint32_t d = tid;
    uint32_t prefix = 0;
    if (tile > 0) {
      int32_t j = (int32_t)tile - 1;
      uint32_t spins = 0;
      while (j >= 0) {
        const uint32_t w =
            __hip_atomic_load(&status[(size_t)j * R + d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t flag = w & ~kStatusCountMask;
        if (flag == 0) {
          if (++spins > kSpinLimit) {
            atomicOr(err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        prefix += w & kStatusCountMask;
        if (flag == kStatusPrefix) break;
        --j;
      }
      __hip_atomic_store(&status[(size_t)tile * R + d], kStatusPrefix | (prefix + count), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    sm.global_off[d] = digit_base[d] + prefix;
  }
  __syncthreads();

  // ---- reorder the tile in LDS by digit
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const uint32_t pos = wave * (KPT * kWave) + j * kWave + lane;
    if (pos < tile_n) {
      const uint32_t d = (uint32_t)(k[j] >> shift) & (R - 1);
      const uint32_t at = sm.local_off[d] + sm.wave_hist[wave][d] + rank[j];
      if (at < kTile) {
        sm.keys[at] = k[j];
        sm.idx[at] = v[j];
      }
    }
  }
  __syncthreads();

  // ---- write digit runs contiguously
  for (uint32_t p = tid; p < tile_n; p += kSortThreads) {
    const K key = sm.keys[p];
    const uint32_t d = (uint32_t)(key >> shift) & (R - 1);
    const uint32_t out = sm.global_off[d] + (p - sm.local_off[d]);
    if (out < n) {  // always true when the histograms are consistent
      keys_out[out] = key;
      idx_out[out] = sm.idx[p];
    }
  }
}

struct Layout {
  size_t keys_alt, idx_alt, hist, counters, status, total;
  uint32_t passes, tile, status_stride;
};

Layout layout_for(int64_t n_max, uint32_t key_bits, uint32_t db, uint32_t kpt) {
  Layout L{};
  const size_t kb = key_bits / 8;
  L.passes = (key_bits + db - 1) / db;
  L.tile = kSortThreads * kpt;
  const size_t tiles = (size_t)((n_max + L.tile - 1) / L.tile) + 1;
  const size_t R = (size_t)1 << db;
  L.status_stride = (uint32_t)(tiles * R);
  size_t off = 0;
  L.keys_alt = off; off = align_up(off + kb * (size_t)n_max, 256);
  L.idx_alt = off; off = align_up(off + 4 * (size_t)n_max, 256);
  L.hist = off; off = align_up(off + 4 * L.passes * R, 256);
  L.counters = off; off = align_up(off + 4 * (L.passes + 1), 256);  // tile counters, then the error word
  L.status = off; off = align_up(off + 4 * (size_t)L.passes * L.status_stride, 256);
  L.total = off;
  return L;
}

template <typename K, int DB, int KPT>
rr_status sort_impl(K* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, char* ws, const Layout& L,
                    hipStream_t st) {
  constexpr uint32_t R = 1u << DB;
  K* kalt = reinterpret_cast<K*>(ws + L.keys_alt);
  uint32_t* ialt = reinterpret_cast<uint32_t*>(ws + L.idx_alt);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  uint32_t* counters = reinterpret_cast<uint32_t*>(ws + L.counters);
  uint32_t* err = counters + L.passes;
  uint32_t* status = reinterpret_cast<uint32_t*>(ws + L.status);
  const uint32_t n = (uint32_t)n_max;
  const uint32_t tiles = (n + L.tile - 1) / L.tile;

  hipLaunchKernelGGL(k_sort_init, dim3(1), dim3(256), 0, st, hist, L.passes * R, counters, L.passes + 1);
  const uint32_t hist_blocks = std::max(1u, std::min(tiles, 2048u));
  hipLaunchKernelGGL((k_sort_hist<K, DB>), dim3(hist_blocks), dim3(kSortThreads), 0, st, keys, count_dev, n,
                     L.passes, hist, status, L.tile, L.status_stride);
  hipLaunchKernelGGL((k_sort_scan<DB>), dim3(1), dim3(kSortThreads), 0, st, hist, L.passes);
  K* src_k = keys;
  uint32_t* src_i = idx;
  K* dst_k = kalt;
  uint32_t* dst_i = ialt;
  for (uint32_t p = 0; p < L.passes; ++p) {
    hipLaunchKernelGGL((k_sort_pass<K, DB, KPT>), dim3(tiles), dim3(kSortThreads), 0, st, src_k, src_i, dst_k,
                       dst_i, count_dev, n, p * DB, hist + p * R, status + (size_t)p * L.status_stride,
                       counters + p, err);
    std::swap(src_k, dst_k);
    std::swap(src_i, dst_i);
  }
  RR_LAUNCH_CHECK();
  // an even pass count leaves the result in the caller's buffers
  return RR_OK;
}

}  // namespace

bool sort_config_supported(uint32_t key_bits, uint32_t digit_bits, uint32_t kpt) {
  return (key_bits == 32 || key_bits == 64) && (digit_bits == 4 || digit_bits == 8) && (kpt == 8 || kpt == 16);
}

size_t sort_workspace_bytes(int64_t n_max, uint32_t key_bits, uint32_t digit_bits, uint32_t kpt) {
  return layout_for(n_max, key_bits, digit_bits, kpt).total;
}

size_t sort_workspace_bytes_any(int64_t n_max, uint32_t key_bits) {
  size_t m = 0;
  for (uint32_t db : {4u, 8u})
    for (uint32_t kpt : {8u, 16u}) m = std::max(m, sort_workspace_bytes(n_max, key_bits, db, kpt));
  return m;
}

rr_status launch_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                      uint32_t db, uint32_t kpt, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!sort_config_supported(key_bits, db, kpt)) return RR_ERR_UNSUPPORTED;
  const Layout L = layout_for(n_max, key_bits, db, kpt);
  if (ws_bytes < L.total) return RR_ERR_WORKSPACE_TOO_SMALL;
  char* w = reinterpret_cast<char*>(ws);
#define RR_SORT_CASE(KT, DBV, KPTV)                                                                   \
  if (sizeof(KT) * 8 == key_bits && db == DBV && kpt == KPTV)                                       \
    return sort_impl<KT, DBV, KPTV>(reinterpret_cast<KT*>(keys), idx, n_max, count_dev, w, L, st);
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

}  // namespace rr
