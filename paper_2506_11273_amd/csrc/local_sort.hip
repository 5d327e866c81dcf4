// Local (block-wise) sort of (key, index) pairs (Section 3.2: the keys may
// be sorted within segments of consecutive keys instead of globally, which
// is cheaper but leaves the ray set less coherent).  Every run of B
// consecutive pairs (B = 1024, 2048 or 4096; the last run may be shorter)
// is sorted on its own, stably by key, entirely in LDS: one workgroup per
// run loads it once into registers, runs all 8-bit LSD digit passes (wave64
// ballot ranking in (wave, slot, lane) order, digit offsets from a scan of
// the per-wave counts, scatter into one LDS buffer, read back), and writes
// it once.  Positions past the run's end hold all-ones keys, which sort
// after every real key (stably after real all-ones keys) and are not
// written.
#include "common.hpp"
#include "wave.hpp"

namespace rr {
namespace {

constexpr int kLsThreads = 1024;
constexpr int kLsWaves = kLsThreads / kWave;
constexpr int kRadix = 256;

template <typename K, int B>
struct LocalSmem {
  K keys[B];
  uint32_t idx[B];
  uint32_t wave_hist[kLsWaves][kRadix];
  uint32_t base[kRadix];
  uint32_t scan[kRadix / kWave];
};

template <typename K, int B>
__global__ __launch_bounds__(kLsThreads) void k_local_sort(K* __restrict__ keys, uint32_t* __restrict__ idx,
                                                          uint32_t n_max, const uint32_t* count_dev,
                                                          uint32_t passes) {
  constexpr int KPT = B / kLsThreads;
  __shared__ LocalSmem<K, B> sm;
  const uint32_t n = count_dev ? min(*count_dev, n_max) : n_max;
  const uint32_t first = blockIdx.x * (uint32_t)B;
  if (first >= n) return;  // block-uniform
  const uint32_t cnt = min((uint32_t)B, n - first);
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;

  K k[KPT];
  uint32_t v[KPT], rank[KPT];
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const uint32_t pos = wave * (KPT * kWave) + j * kWave + lane;
    k[j] = pos < cnt ? keys[first + pos] : ~(K)0;
    v[j] = pos < cnt ? idx[first + pos] : 0xFFFFFFFFu;
  }
  for (uint32_t pass = 0; pass < passes; ++pass) {
    const uint32_t shift = pass * 8;
    for (uint32_t i = tid; i < kLsWaves * kRadix; i += kLsThreads) (&sm.wave_hist[0][0])[i] = 0;
    __syncthreads();
    // ---- rank within the wave, in (slot, lane) order: the lowest lane of
    // each group of equal digits adds the group's size to the wave's count
    // with an LDS atomic (the leaders of one slot hold distinct digits, and
    // a wave's LDS operations take effect in order); the group's lanes take
    // the returned count once every slot has been issued
    uint32_t old[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const uint32_t d = (uint32_t)(k[j] >> shift) & (kRadix - 1);
      const uint64_t peers = match_digit<8>(d, ~0ull);
      const uint32_t leader = (uint32_t)__builtin_ctzll(peers);
      rank[j] = lanes_below(peers) | (leader << 16);
      old[j] = 0;
      if (lane == leader) old[j] = atomicAdd(&sm.wave_hist[wave][d], (uint32_t)__popcll(peers));
    }
#pragma unroll
    for (int j = 0; j < KPT; ++j) rank[j] = (rank[j] & 0xFFFFu) + __shfl(old[j], (int)(rank[j] >> 16), kWave);
    __syncthreads();
    // ---- per digit: offsets of the waves, then the digits' bases
    if (tid < kRadix) {
      uint32_t c = 0;
#pragma unroll
      for (int w = 0; w < kLsWaves; ++w) {
        const uint32_t t = sm.wave_hist[w][tid];
        sm.wave_hist[w][tid] = c;
        c += t;
      }
      // exclusive scan of the digit totals over the first 256 threads
      uint32_t x = c;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, kWave);
        if ((int)lane >= off) x += y;
      }
      if (lane == kWave - 1) sm.scan[wave] = x;
      sm.base[tid] = x - c;  // exclusive within the wave for now
    }
    __syncthreads();
    if (tid < kRadix) {
      uint32_t add = 0;
#pragma unroll
      for (int w = 0; w < kRadix / kWave; ++w) add += (uint32_t)w < wave ? sm.scan[w] : 0u;
      sm.base[tid] += add;
    }
    __syncthreads();
    // ---- scatter into LDS in digit order, then read back wave-striped
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const uint32_t d = (uint32_t)(k[j] >> shift) & (kRadix - 1);
      const uint32_t at = sm.base[d] + sm.wave_hist[wave][d] + rank[j];
      sm.keys[at] = k[j];
      sm.idx[at] = v[j];
    }
    __syncthreads();
    if (pass + 1 < passes) {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const uint32_t pos = wave * (KPT * kWave) + j * kWave + lane;
        k[j] = sm.keys[pos];
        v[j] = sm.idx[pos];
      }
    }
  }
  // ---- write the sorted run (the padding sorts to the end)
  for (uint32_t p = tid; p < cnt; p += kLsThreads) {
    keys[first + p] = sm.keys[p];
    idx[first + p] = sm.idx[p];
  }
}

template <typename K, int B>
void launch_local(void* keys, uint32_t* idx, uint32_t n_max, const uint32_t* count_dev, uint32_t passes,
                  hipStream_t st) {
  const uint32_t blocks = (n_max + B - 1) / B;
  hipLaunchKernelGGL((k_local_sort<K, B>), dim3(blocks), dim3(kLsThreads), 0, st, reinterpret_cast<K*>(keys), idx,
                     n_max, count_dev, passes);
}

}  // namespace

bool local_sort_supported(uint32_t key_bits, uint32_t block) {
  return (key_bits == 32 || key_bits == 64) && (block == 1024 || block == 2048 || block == 4096);
}

rr_status launch_local_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                            uint32_t block, hipStream_t st) {
  if (!local_sort_supported(key_bits, block)) return RR_ERR_UNSUPPORTED;
  if (n_max == 0) return RR_OK;
  const uint32_t n = (uint32_t)n_max, passes = key_bits / 8;
  if (key_bits == 32) {
    if (block == 1024) launch_local<uint32_t, 1024>(keys, idx, n, count_dev, passes, st);
    else if (block == 2048) launch_local<uint32_t, 2048>(keys, idx, n, count_dev, passes, st);
    else launch_local<uint32_t, 4096>(keys, idx, n, count_dev, passes, st);
  } else {
    if (block == 1024) launch_local<uint64_t, 1024>(keys, idx, n, count_dev, passes, st);
    else if (block == 2048) launch_local<uint64_t, 2048>(keys, idx, n, count_dev, passes, st);
    else launch_local<uint64_t, 4096>(keys, idx, n, count_dev, passes, st);
  }
  RR_LAUNCH_CHECK();
  return RR_OK;
}

}  // namespace rr
