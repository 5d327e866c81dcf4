// Sort-key computation (Section 3.1, Figure "codes") with optional stable
// compaction of live rays, and the length table of Two Point Adaptive
// (Section 3.1.6).
//
// Each key is the Morton-style interleave of quantised ray coordinates: an
// origin-direction key (Section 3.1.2) puts the origin bits above the
// direction bits, the Two Point key (Section 3.1.5) interleaves origin and
// estimated termination point, the latter at a fixed length of a ratio of the
// largest scene extent (Section 3.1.6).  Bits are placed with the classic
// "spread by 3" magic-mask sequences rather than a per-slot loop: a component
// with b slots at stride s has its bit i at key bit s*i + shift.
//
// The kernel is HBM bound: 32 bytes of ray in, 8 or 12 bytes out per ray.
#include "common.hpp"
#include "keys_dev.hpp"

#pragma clang fp contract(off)

namespace rr {

namespace {

// The figure's other layouts as runs of slots, most significant first.  A
// run cycles its vector's components; vector 0 origin, 1 direction, 2 zero
// slots, 3 octahedral (u, v).
struct Run {
  int vec, n;
};

// Places each component's slots and splits them into fields of equally
// spaced slots.
rr_status general_plan(int kind, KeyPlan* P) {
  static const Run kOrigin[] = {{0, 32}};
  static const Run kCosta[] = {{1, 8}, {0, 24}};
  static const Run kAila[] = {{0, 3}, {2, 3}, {0, 3}, {2, 3}, {0, 3}, {2, 3}, {0, 3}, {1, 3}, {0, 3}, {1, 3}, {0, 2}};
  static const Run kAilaCompact[] = {{0, 12}, {1, 3}, {0, 3}, {1, 3}, {0, 3}, {1, 3}, {0, 3}, {1, 2}};
  static const Run kOctahedron[] = {{0, 15}, {3, 2}, {0, 3}, {3, 2}, {0, 3}, {3, 2}, {0, 3}, {3, 2}};
  const Run* runs = nullptr;
  int nruns = 0;
  switch (kind) {
    case RR_KEY_ORIGIN: runs = kOrigin; nruns = 1; break;
    case RR_KEY_DIRECTION_ORIGIN: runs = kCosta; nruns = 2; break;
    case RR_KEY_AILA: runs = kAila; nruns = 11; break;
    case RR_KEY_AILA_COMPACT: runs = kAilaCompact; nruns = 8; break;
    case RR_KEY_OCTAHEDRON: runs = kOctahedron; nruns = 8; break;
    default: return RR_ERR_INVALID_ARGUMENT;
  }
  int pos[6][32];  // key bit of each component's slots, its MSB first
  int npos[6] = {0, 0, 0, 0, 0, 0};
  int slot = 31;
  for (int r = 0; r < nruns; ++r) {
    const int ncomp = runs[r].vec == 3 ? 2 : 3;
    for (int i = 0; i < runs[r].n; ++i, --slot) {
      if (runs[r].vec == 2) continue;
      const int c = (runs[r].vec == 0 ? 0 : 3) + i % ncomp;
      pos[c][npos[c]++] = slot;
    }
  }
  if (slot != -1) return RR_ERR_INVALID_ARGUMENT;
  P->nfields = 0;
  for (int c = 0; c < 6; ++c) {
    const int b = npos[c];
    P->scale[c] = b ? (float)(1u << b) : 1.0f;
    P->qmax[c] = b ? (1u << b) - 1u : 0u;
    P->shift[c] = 0;
    for (int k = 0; k < b;) {
      const int stride = k + 1 < b ? pos[c][k] - pos[c][k + 1] : 1;
      int e = k + 1;
      while (e < b && pos[c][e - 1] - pos[c][e] == stride) ++e;
      if (P->nfields == kMaxKeyFields) return RR_ERR_INVALID_ARGUMENT;
      KeyField& F = P->field[P->nfields++];
      F.comp = (uint8_t)c;
      F.cnt = (uint8_t)(e - k);
      F.stride = (uint8_t)stride;
      F.src_shift = (uint8_t)(b - e);
      F.dst_shift = (uint8_t)pos[c][e - 1];
      k = e;
    }
  }
  return RR_OK;
}

}  // namespace

rr_status make_key_plan(const rr_key_params* p, KeyPlan* out) {
  if (!p || !out) return RR_ERR_INVALID_ARGUMENT;
  if (p->key_bits != 32 && p->key_bits != 64) return RR_ERR_INVALID_ARGUMENT;
  if (p->kind < RR_KEY_ORIGIN_DIRECTION || p->kind > RR_KEY_TWO_POINT_REAL) return RR_ERR_INVALID_ARGUMENT;
  const bool general = p->kind >= RR_KEY_ORIGIN && p->kind <= RR_KEY_OCTAHEDRON;
  if (general && p->key_bits != 32) return RR_ERR_UNSUPPORTED;
  const bool needs_aux = p->kind == RR_KEY_TWO_POINT_ADAPTIVE || p->kind == RR_KEY_TWO_POINT_REAL;
  if (needs_aux && !p->aux) return RR_ERR_INVALID_ARGUMENT;
  KeyPlan P{};
  const int K = (int)p->key_bits;
  float ext[3];
  for (int k = 0; k < 3; ++k) {
    ext[k] = p->box_hi[k] - p->box_lo[k];
    P.lo[k] = p->box_lo[k];
    P.inv[k] = ext[k] > 0.0f ? 1.0f / ext[k] : 0.0f;
  }
  float E = ext[0];
  if (ext[1] > E) E = ext[1];
  if (ext[2] > E) E = ext[2];
  P.len = p->term_ratio * E;
  P.E = E;
  P.s24 = 16777216.0f / E;
  P.kind = p->kind;
  P.key64 = K == 64;
  P.aux = needs_aux ? p->aux : nullptr;

  // A field of S slots starting at key bit `base`, cycling over `cyc`
  // components: component j owns ceil((S - j) / cyc) slots; its slot m
  // (from the field's top) sits at base + S - 1 - j - cyc*m and carries the
  // component's bit b - 1 - m, hence bit i lands at cyc*i + shift.
  auto place = [&](int first_comp, int ncomp, int cyc, int S, int base) {
    for (int j = 0; j < ncomp; ++j) {
      int c = first_comp + j;
      int b = S > j ? (S - j + cyc - 1) / cyc : 0;
      if (b <= 0) {
        P.scale[c] = 1.0f;
        P.qmax[c] = 0;
        P.shift[c] = 0;
        continue;
      }
      P.scale[c] = (float)(1u << b);
      P.qmax[c] = (1u << b) - 1u;
      P.shift[c] = base + S - 1 - j - cyc * (b - 1);
    }
  };
  if (p->kind == RR_KEY_ORIGIN_DIRECTION) {
    int ob = p->origin_bits ? (int)p->origin_bits : (K == 32 ? 22 : 44);
    if (ob > K) return RR_ERR_INVALID_ARGUMENT;
    place(0, 3, 3, ob, K - ob);
    place(3, 3, 3, K - ob, 0);
  } else if (general) {
    rr_status st = general_plan(p->kind, &P);
    if (st != RR_OK) return st;
  } else {
    // the six components cycle together over the whole key
    int S = K;
    for (int j = 0; j < 6; ++j) {
      int b = (S - j + 5) / 6;
      P.scale[j] = (float)(1u << b);
      P.qmax[j] = (1u << b) - 1u;
      P.shift[j] = S - 1 - j - 6 * (b - 1);
    }
  }
  // spread3 interleaves components of at most 21 bits
  for (int c = 0; c < 6; ++c)
    if (P.qmax[c] >= (1u << 21)) return RR_ERR_UNSUPPORTED;
  *out = P;
  return RR_OK;
}

namespace {

constexpr int kKeyBlock = 256;
constexpr int kCompactPer = 4;
constexpr int kCompactTile = kKeyBlock * kCompactPer;  // rays per compaction block

template <int KIND, typename K>
__global__ __launch_bounds__(kKeyBlock) void k_keys_dense(const float4* __restrict__ rays, uint32_t n, KeyPlan P,
                                                          K* __restrict__ keys, uint32_t* __restrict__ idx,
                                                          uint32_t* count_out) {
  const uint32_t i = blockIdx.x * kKeyBlock + threadIdx.x;
  if (i == 0 && count_out) *count_out = n;
  if (i >= n) return;
  const float4 a = rays[2 * (size_t)i];
  const float4 b = rays[2 * (size_t)i + 1];
  keys[i] = (K)ray_key<KIND>(a, b, P, i);
  idx[i] = i;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Live rays per block of kCompactTile slots.
__global__ __launch_bounds__(kKeyBlock) void k_alive_count(const uint8_t* __restrict__ alive, uint32_t n,
                                                           uint32_t* __restrict__ block_counts) {
  __shared__ uint32_t s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kCompactTile;
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < kCompactPer; ++r) {
    const uint32_t i = base + r * kKeyBlock + threadIdx.x;
    c += (i < n && alive[i]) ? 1u : 0u;
  }
  // wave sum by ballots over the 3 bits of c (c <= 4)
  uint32_t w = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) w += (uint32_t)__popcll(__ballot((c >> b) & 1u)) << b;
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&s_sum, w);
  __syncthreads();
  if (threadIdx.x == 0) block_counts[blockIdx.x] = s_sum;
}

// Exclusive scan of the block counts in place (one block of 1024 threads);
// the total goes to *count_out.
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t* __restrict__ v, uint32_t nblocks,
                                                      uint32_t* __restrict__ count_out) {
  __shared__ uint32_t s[1024];
  uint32_t running = 0;
  for (uint32_t base = 0; base < nblocks; base += 1024) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t x = i < nblocks ? v[i] : 0u;
    s[threadIdx.x] = x;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
      const uint32_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nblocks) v[i] = running + s[threadIdx.x] - x;
    running += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0 && count_out) *count_out = running;
}

// Keys (or only indices when WITH_KEYS is false) of the live rays, written
// at their compacted positions: ascending original index.
template <int KIND, typename K, bool WITH_KEYS>
__global__ __launch_bounds__(kKeyBlock) void k_keys_compact(const float4* __restrict__ rays,
                                                            const uint8_t* __restrict__ alive, uint32_t n, KeyPlan P,
                                                            const uint32_t* __restrict__ block_off,
                                                            K* __restrict__ keys, uint32_t* __restrict__ idx) {
  __shared__ uint32_t s_w[kKeyBlock / kWave];
  const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint32_t base = blockIdx.x * kCompactTile;
  uint32_t running = block_off[blockIdx.x];
  for (int r = 0; r < kCompactPer; ++r) {
    const uint32_t i = base + r * kKeyBlock + threadIdx.x;
    const bool live = i < n && alive[i];
    const uint64_t m = __ballot(live);
    if (lane == 0) s_w[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kKeyBlock / kWave; ++w) {
      const uint32_t c = s_w[w];
      before += w < wave ? c : 0u;
      total += c;
    }
    if (live) {
      const uint32_t pos = running + before + lanes_below(m);
      if constexpr (WITH_KEYS) {
        const float4 a = rays[2 * (size_t)i];
        const float4 b = rays[2 * (size_t)i + 1];
        keys[pos] = (K)ray_key<KIND>(a, b, P, i);
      }
      idx[pos] = i;
    }
    running += total;
    __syncthreads();
  }
}

template <int KIND, typename K>
rr_status keys_impl(const rr_ray* rays, int64_t n, const uint8_t* alive, const KeyPlan& P, K* keys, uint32_t* idx,
                    uint32_t* count_out, uint32_t* block_scratch, hipStream_t st) {
  const float4* r4 = reinterpret_cast<const float4*>(rays);
  if (!alive) {
    const uint32_t blocks = (uint32_t)((n + kKeyBlock - 1) / kKeyBlock);
    hipLaunchKernelGGL((k_keys_dense<KIND, K>), dim3(blocks), dim3(kKeyBlock), 0, st, r4, (uint32_t)n, P, keys, idx,
                       count_out);
    RR_LAUNCH_CHECK();
    return RR_OK;
  }
  const uint32_t nb = (uint32_t)((n + kCompactTile - 1) / kCompactTile);
  hipLaunchKernelGGL(k_alive_count, dim3(nb), dim3(kKeyBlock), 0, st, alive, (uint32_t)n, block_scratch);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, block_scratch, nb, count_out);
  hipLaunchKernelGGL((k_keys_compact<KIND, K, true>), dim3(nb), dim3(kKeyBlock), 0, st, r4, alive, (uint32_t)n, P,
                     block_scratch, keys, idx);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

}  // namespace

size_t keys_scratch_bytes(int64_t n) {
  return align_up(sizeof(uint32_t) * (size_t)((n + kCompactTile - 1) / kCompactTile + 1), 256);
}

rr_status launch_keys(const rr_ray* rays, int64_t n, const uint8_t* alive, const KeyPlan& P, void* keys,
                      uint32_t* idx, uint32_t* count_out, void* block_scratch, hipStream_t st) {
  uint32_t* bs = reinterpret_cast<uint32_t*>(block_scratch);
  switch (key_family(P.kind)) {
    case 1:
      if (P.key64) return keys_impl<1, uint64_t>(rays, n, alive, P, (uint64_t*)keys, idx, count_out, bs, st);
      return keys_impl<1, uint32_t>(rays, n, alive, P, (uint32_t*)keys, idx, count_out, bs, st);
    case 2:
      if (P.key64) return keys_impl<2, uint64_t>(rays, n, alive, P, (uint64_t*)keys, idx, count_out, bs, st);
      return keys_impl<2, uint32_t>(rays, n, alive, P, (uint32_t*)keys, idx, count_out, bs, st);
    default:
      return keys_impl<3, uint32_t>(rays, n, alive, P, (uint32_t*)keys, idx, count_out, bs, st);
  }
}

namespace {

__global__ __launch_bounds__(kKeyBlock) void k_length_init(rr_length_cell* __restrict__ table, uint64_t sum0) {
  const uint32_t i = blockIdx.x * kKeyBlock + threadIdx.x;
  if (i < kLengthCells) table[i] = rr_length_cell{sum0, 1u, 0u};
}

// Adds the traced length of each hit to its ray's cell: fixed point in
// units of E / 2^24, truncated, clamped to [0, 2^40].
__global__ __launch_bounds__(kKeyBlock) void k_length_accumulate(rr_length_cell* __restrict__ table,
                                                                 const float4* __restrict__ rays,
                                                                 const uint32_t* __restrict__ idx,
                                                                 const float4* __restrict__ hits, uint32_t n_max,
                                                                 const uint32_t* count_dev, KeyPlan P) {
  const uint32_t n = count_dev ? min(*count_dev, n_max) : n_max;
  const uint32_t i = blockIdx.x * kKeyBlock + threadIdx.x;
  if (i >= n) return;
  const float4 h = hits[i];
  if (__float_as_int(h.y) < 0) return;
  const uint32_t r = idx ? idx[i] : i;
  const float4 a = rays[2 * (size_t)r];
  const float4 b = rays[2 * (size_t)r + 1];
  const float x = h.x * P.s24;
  const uint64_t q = !(x > 0.0f) ? 0ull : (x > 1099511627776.0f ? 1099511627776ull : (uint64_t)x);
  rr_length_cell* c = &table[cell_code(a, b, P)];
  atomicAdd(reinterpret_cast<unsigned long long*>(&c->sum), (unsigned long long)q);
  atomicAdd(&c->count, 1u);
}

}  // namespace

rr_status launch_length_init(rr_length_cell* table, const KeyPlan& P, float ratio, hipStream_t st) {
  (void)P;
  const uint64_t sum0 = (uint64_t)(ratio * 16777216.0f);
  hipLaunchKernelGGL(k_length_init, dim3(kLengthCells / kKeyBlock), dim3(kKeyBlock), 0, st, table, sum0);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status launch_length_accumulate(rr_length_cell* table, const rr_ray* rays, const uint32_t* idx,
                                   const rr_hit* hits, int64_t n_max, const uint32_t* count_dev, const KeyPlan& P,
                                   hipStream_t st) {
  if (n_max == 0) return RR_OK;
  const uint32_t blocks = (uint32_t)((n_max + kKeyBlock - 1) / kKeyBlock);
  hipLaunchKernelGGL(k_length_accumulate, dim3(blocks), dim3(kKeyBlock), 0, st, table,
                     reinterpret_cast<const float4*>(rays), idx, reinterpret_cast<const float4*>(hits),
                     (uint32_t)n_max, count_dev, P);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status launch_compact_only(int64_t n, const uint8_t* alive, uint32_t* idx, uint32_t* count_out,
                              void* block_scratch, hipStream_t st) {
  uint32_t* bs = reinterpret_cast<uint32_t*>(block_scratch);
  const uint32_t nb = (uint32_t)((n + kCompactTile - 1) / kCompactTile);
  KeyPlan P{};
  hipLaunchKernelGGL(k_alive_count, dim3(nb), dim3(kKeyBlock), 0, st, alive, (uint32_t)n, bs);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bs, nb, count_out);
  hipLaunchKernelGGL((k_keys_compact<1, uint32_t, false>), dim3(nb), dim3(kKeyBlock), 0, st, nullptr, alive,
                     (uint32_t)n, P, bs, nullptr, idx);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

}  // namespace rr
