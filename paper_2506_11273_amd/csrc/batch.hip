// Batched reordering and tracing: many wavefronts of uneven size (rays of
// different bounces, each segment with its own key method) reordered and
// traced together against one resident scene.
//
// The arithmetic is that of the per-call path (Section 3.1 keys, Section 3.2
// key/index sort and ray gather, Section 4.1 closest-hit trace), applied per
// segment: the sort is segmented, and the gather and trace run once over all
// segments packed back to back.  Every kernel is persistent (a grid sized to
// the device, looping over the work) and reads the batch's sizes and
// pointers from a descriptor table in device memory, so one captured
// hipGraph serves any mix of segment sizes; a run is one descriptor upload
// plus one graph launch.
//
// 32-bit keys of a batch that also holds 64-bit keys are placed in the high
// half of a 64-bit key, which leaves their stable order unchanged; segments
// without a key (RR_KEY_NONE) get key 0 and keep their order.
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "keys_dev.hpp"
#include "rr_batch.h"
#include "sort_seg.hpp"

namespace rr {

struct BatchSeg {
  const float4* rays;
  float4* hits;
  uint32_t* perm;
  uint32_t n, out_off, shift, orig;  // shift: where the key lands in the batch's key word
  KeyPlan plan;                      // plan.kind 0: no key
};

struct BatchHdr {
  uint32_t nseg, total, pad0, pad1;
};

namespace {

constexpr int kBatchBlock = 256;
constexpr int kRing = 4;

// Segment of packed position p: the last segment starting at or before p
// (an empty segment shares its start with the next one and is passed over).
__device__ __forceinline__ uint32_t seg_of_pos(const BatchSeg* segs, uint32_t nseg, uint32_t p) {
  uint32_t lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (segs[mid].out_off <= p) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The same for positions that ascend with the lane (the streaming loops
// below): one wave-uniform search from the first active lane's position,
// then each lane steps over the few segment starts between it and its own.
__device__ __forceinline__ uint32_t seg_of_pos_wave(const BatchSeg* segs, uint32_t nseg, uint32_t p) {
  const uint32_t p0 = __builtin_amdgcn_readfirstlane(p);
  uint32_t s = seg_of_pos(segs, nseg, p0);
  if (p < p0) return seg_of_pos(segs, nseg, p);  // not taken: positions ascend with the lane
  while (s + 1 < nseg && segs[s + 1].out_off <= p) ++s;
  return s;
}

// Runs f(segment) with the segment index wave-uniform when every active
// lane is in the same segment (so its descriptor is read with scalar
// loads), else per lane.
template <typename F>
__device__ __forceinline__ void with_segment(const BatchSeg* segs, uint32_t s, F&& f) {
  const uint32_t su = __builtin_amdgcn_readfirstlane(s);
  if (__ballot(s != su) == 0) f(segs[su]);
  else f(segs[s]);
}

template <typename K>
__global__ __launch_bounds__(kBatchBlock) void k_batch_keys(const BatchHdr* __restrict__ hdr,
                                                            const BatchSeg* __restrict__ segs, K* __restrict__ keys,
                                                            uint32_t* __restrict__ idx) {
  const uint32_t total = hdr->total, nseg = hdr->nseg;
  for (uint32_t p = blockIdx.x * kBatchBlock + threadIdx.x; p < total; p += gridDim.x * kBatchBlock) {
    with_segment(segs, seg_of_pos_wave(segs, nseg, p), [&](const BatchSeg& S) {
      const uint32_t r = p - S.out_off;
      uint64_t key = 0;
      if (S.plan.kind != 0) {
        const float4 a = S.rays[2 * (size_t)r];
        const float4 b = S.rays[2 * (size_t)r + 1];
        key = ray_key_any(a, b, S.plan, r);
        key <<= S.shift;
      }
      keys[p] = (K)key;
      idx[p] = r;
    });
  }
}

// After the segmented sort, position p still lies in its segment's range.
__global__ __launch_bounds__(kBatchBlock) void k_batch_gather(const BatchHdr* __restrict__ hdr,
                                                              const BatchSeg* __restrict__ segs,
                                                              const uint32_t* __restrict__ idx,
                                                              float4* __restrict__ out) {
  const uint32_t total = hdr->total, nseg = hdr->nseg;
  for (uint32_t t = blockIdx.x * kBatchBlock + threadIdx.x; t < 2 * total; t += gridDim.x * kBatchBlock) {
    const uint32_t i = t >> 1, h = t & 1;
    with_segment(segs, seg_of_pos_wave(segs, nseg, i),
                 [&](const BatchSeg& S) { out[2 * (size_t)i + h] = S.rays[2 * (size_t)idx[i] + h]; });
  }
}

__global__ __launch_bounds__(kBatchBlock) void k_batch_out(const BatchHdr* __restrict__ hdr,
                                                           const BatchSeg* __restrict__ segs,
                                                           const uint32_t* __restrict__ idx,
                                                           const float4* __restrict__ hits_sorted) {
  const uint32_t total = hdr->total, nseg = hdr->nseg;
  for (uint32_t p = blockIdx.x * kBatchBlock + threadIdx.x; p < total; p += gridDim.x * kBatchBlock) {
    with_segment(segs, seg_of_pos_wave(segs, nseg, p), [&](const BatchSeg& S) {
      const uint32_t r = idx[p], q = p - S.out_off;
      S.hits[S.orig ? r : q] = hits_sorted[p];
      if (S.perm) S.perm[q] = r;
    });
  }
}

// Grid of the streaming kernels: 8 blocks per CU, queried once (thread-safe
// static initialisation: the server's thread launches batches too).
uint32_t streaming_blocks() {
  static const uint32_t v = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    return (uint32_t)cus * 8;
  }();
  return v;
}

}  // namespace
}  // namespace rr

using namespace rr;

struct rr_batch_s {
  rr_scene scene = nullptr;
  int device = 0;
  int64_t cap = 0;
  int32_t max_seg = 0;
  rr_batch_config cfg{8, 16, kDefaultRefill, RR_TILES_COUNTER, 256};
  char* dev = nullptr;  // one device allocation for everything below
  size_t bytes = 0;
  size_t off_hdr = 0, off_segs = 0, off_shdr = 0, off_ssegs = 0, off_keys = 0, off_idx = 0, off_rays = 0,
         off_hits = 0, off_ws = 0, desc_bytes = 0;
  char* pinned[kRing] = {};  // descriptor staging, reused once its copy has completed
  hipEvent_t staged[kRing] = {};
  bool staged_used[kRing] = {};
  int ring = 0;
  hipStream_t capture = nullptr;
  struct Graph {
    uint32_t kb, db, kpt, refill, order, block;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  std::mutex mu;
};

namespace {

size_t batch_sort_ws(int64_t cap, int32_t max_seg) {
  size_t m = 0;
  for (uint32_t kb : {32u, 64u})
    for (uint32_t db : {4u, 8u})
      for (uint32_t kpt : {8u, 16u}) m = std::max(m, seg_layout(cap, (uint32_t)max_seg, kb, db, kpt).total);
  return m;
}

bool valid_cfg(const rr_batch_config& c) {
  return (c.digit_bits == 4 || c.digit_bits == 8) && (c.keys_per_thread == 8 || c.keys_per_thread == 16) &&
         c.refill >= 1 && c.refill <= 64 && (c.tile_order == RR_TILES_COUNTER || c.tile_order == RR_TILES_FIXED) &&
         (c.trace_block == 128 || c.trace_block == 256 || c.trace_block == 512);
}

// Enqueues the whole batched path on st (eagerly or into a capture).
rr_status enqueue(rr_batch b, uint32_t kb, const rr_batch_config& c, hipStream_t st) {
  char* d = b->dev;
  const BatchHdr* hdr = reinterpret_cast<const BatchHdr*>(d + b->off_hdr);
  const BatchSeg* segs = reinterpret_cast<const BatchSeg*>(d + b->off_segs);
  SortHdr* shdr = reinterpret_cast<SortHdr*>(d + b->off_shdr);
  SortSeg* ssegs = reinterpret_cast<SortSeg*>(d + b->off_ssegs);
  uint32_t* idx = reinterpret_cast<uint32_t*>(d + b->off_idx);
  float4* srays = reinterpret_cast<float4*>(d + b->off_rays);
  float4* shits = reinterpret_cast<float4*>(d + b->off_hits);
  const uint32_t grid = streaming_blocks();
  if (kb == 64)
    hipLaunchKernelGGL(k_batch_keys<uint64_t>, dim3(grid), dim3(kBatchBlock), 0, st, hdr, segs,
                       reinterpret_cast<uint64_t*>(d + b->off_keys), idx);
  else
    hipLaunchKernelGGL(k_batch_keys<uint32_t>, dim3(grid), dim3(kBatchBlock), 0, st, hdr, segs,
                       reinterpret_cast<uint32_t*>(d + b->off_keys), idx);
  RR_LAUNCH_CHECK();
  const SegLayout L = seg_layout(b->cap, (uint32_t)b->max_seg, kb, c.digit_bits, c.keys_per_thread);
  rr_status r = launch_seg_sort(d + b->off_keys, idx, L, d + b->off_ws, shdr, ssegs, nullptr, (uint32_t)b->cap, kb,
                                c.digit_bits, c.keys_per_thread, c.tile_order == RR_TILES_COUNTER, st);
  if (r != RR_OK) return r;
  hipLaunchKernelGGL(k_batch_gather, dim3(grid), dim3(kBatchBlock), 0, st, hdr, segs, idx, srays);
  RR_LAUNCH_CHECK();
  const uint32_t* total = reinterpret_cast<const uint32_t*>(d + b->off_hdr + offsetof(BatchHdr, total));
  r = launch_trace_refill(b->scene->d, reinterpret_cast<const rr_ray*>(srays), nullptr, b->cap, total,
                          reinterpret_cast<rr_hit*>(shits), c.refill, st, c.trace_block);
  if (r != RR_OK) return r;
  hipLaunchKernelGGL(k_batch_out, dim3(grid), dim3(kBatchBlock), 0, st, hdr, segs, idx, shits);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status graph_for(rr_batch b, uint32_t kb, const rr_batch_config& c, hipGraphExec_t* out) {
  for (auto& g : b->graphs)
    if (g.kb == kb && g.db == c.digit_bits && g.kpt == c.keys_per_thread && g.refill == c.refill &&
        g.order == c.tile_order && g.block == c.trace_block) {
      *out = g.exec;
      return RR_OK;
    }
  // one-time host queries must not happen inside the capture
  sort_warm(kb, c.digit_bits, c.keys_per_thread);
  trace_warm();
  (void)streaming_blocks();
  if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return RR_ERR_DEVICE;
  rr_status r = enqueue(b, kb, c, b->capture);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->capture, &g);
  if (r != RR_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return r != RR_OK ? r : RR_ERR_DEVICE;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return RR_ERR_DEVICE;
  b->graphs.push_back({kb, c.digit_bits, c.keys_per_thread, c.refill, c.tile_order, c.trace_block, exec});
  *out = exec;
  return RR_OK;
}

bool is_dev(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Validates the segments and fills host descriptor staging h; returns the
// batch key width.
rr_status stage(rr_batch b, const rr_segment* segs, int32_t nseg, uint32_t flags, const rr_batch_config& c,
                char* h, uint32_t* kb_out) {
  if (nseg < 0 || nseg > b->max_seg || (nseg > 0 && !segs)) return RR_ERR_INVALID_ARGUMENT;
  uint32_t kb = 32;
  int64_t total = 0;
  for (int32_t s = 0; s < nseg; ++s) {
    const rr_segment& g = segs[s];
    if (g.n < 0) return RR_ERR_INVALID_ARGUMENT;
    if (g.n > 0) {
      if (!is_dev(g.rays) || !is_dev(g.hits) || (reinterpret_cast<uintptr_t>(g.rays) & 15) ||
          (reinterpret_cast<uintptr_t>(g.hits) & 15))
        return RR_ERR_INVALID_ARGUMENT;
      if (g.perm && (!is_dev(g.perm) || (reinterpret_cast<uintptr_t>(g.perm) & 3))) return RR_ERR_INVALID_ARGUMENT;
    }
    if (g.key.kind != RR_KEY_NONE) {
      if (g.key.key_bits != 32 && g.key.key_bits != 64) return RR_ERR_INVALID_ARGUMENT;
      if (g.key.key_bits == 64) kb = 64;
    }
    total += g.n;
  }
  if (total > b->cap) return RR_ERR_BUDGET;
  const uint32_t tile = sort_tile_keys(c.keys_per_thread);
  BatchHdr H{(uint32_t)nseg, (uint32_t)total, 0u, 0u};
  BatchSeg* bs = reinterpret_cast<BatchSeg*>(h + b->off_segs);
  SortSeg* ss = reinterpret_cast<SortSeg*>(h + b->off_ssegs);
  uint32_t out = 0, toff = 0;
  for (int32_t s = 0; s < nseg; ++s) {
    const rr_segment& g = segs[s];
    BatchSeg B{};
    B.rays = reinterpret_cast<const float4*>(g.rays);
    B.hits = reinterpret_cast<float4*>(g.hits);
    B.perm = g.perm;
    B.n = (uint32_t)g.n;
    B.out_off = out;
    B.orig = (flags & RR_HITS_ORIGINAL_ORDER) ? 1u : 0u;
    if (g.key.kind != RR_KEY_NONE) {
      rr_status r = make_key_plan(&g.key, &B.plan);
      if (r != RR_OK) return r;
      if (B.plan.aux && (!is_dev(B.plan.aux) || (reinterpret_cast<uintptr_t>(B.plan.aux) & 15)))
        return RR_ERR_INVALID_ARGUMENT;
      B.shift = (kb == 64 && g.key.key_bits == 32) ? 32u : 0u;
    }
    std::memcpy(&bs[s], &B, sizeof B);
    const uint32_t nt = (uint32_t)((g.n + tile - 1) / tile);
    const SortSeg S{out, (uint32_t)g.n, toff, nt};
    std::memcpy(&ss[s], &S, sizeof S);
    out += (uint32_t)g.n;
    toff += nt;
  }
  const SortHdr SH{(uint32_t)nseg, toff, out, 0u};
  std::memcpy(h + b->off_hdr, &H, sizeof H);
  std::memcpy(h + b->off_shdr, &SH, sizeof SH);
  *kb_out = kb;
  return RR_OK;
}

void free_batch(rr_batch b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  for (int k = 0; k < kRing; ++k) {
    if (b->staged[k]) (void)hipEventDestroy(b->staged[k]);
    if (b->pinned[k]) (void)hipHostFree(b->pinned[k]);
  }
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->dev) (void)hipFree(b->dev);
  delete b;
}

}  // namespace

extern "C" {

rr_status rr_batch_create(rr_scene s, int64_t max_rays, int32_t max_segments, const rr_batch_config* cfg,
                          rr_batch* out) {
  if (!out) return RR_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!s || max_rays <= 0 || max_rays >= RR_MAX_RAYS || max_segments <= 0 || max_segments > 4096)
    return RR_ERR_INVALID_ARGUMENT;
  if (cfg && !valid_cfg(*cfg)) return RR_ERR_INVALID_ARGUMENT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->d.device) return RR_ERR_INVALID_ARGUMENT;
  rr_batch b = new (std::nothrow) rr_batch_s;
  if (!b) return RR_ERR_OUT_OF_MEMORY;
  b->scene = s;
  b->device = dev;
  b->cap = max_rays;
  b->max_seg = max_segments;
  if (cfg) b->cfg = *cfg;
  size_t off = 0;
  b->off_hdr = off; off = align_up(off + sizeof(BatchHdr), 256);
  b->off_segs = off; off = align_up(off + sizeof(BatchSeg) * (size_t)max_segments, 256);
  b->off_shdr = off; off = align_up(off + sizeof(SortHdr), 256);
  b->off_ssegs = off; off = align_up(off + sizeof(SortSeg) * (size_t)max_segments, 256);
  b->desc_bytes = off;
  b->off_keys = off; off = align_up(off + 8 * (size_t)max_rays, 256);
  b->off_idx = off; off = align_up(off + 4 * (size_t)max_rays, 256);
  b->off_rays = off; off = align_up(off + sizeof(rr_ray) * (size_t)max_rays, 256);
  b->off_hits = off; off = align_up(off + sizeof(rr_hit) * (size_t)max_rays, 256);
  b->off_ws = off; off = align_up(off + batch_sort_ws(max_rays, max_segments), 256);
  b->bytes = off;
  rr_status st = RR_OK;
  if (hipMalloc(&b->dev, b->bytes) != hipSuccess) st = RR_ERR_OUT_OF_MEMORY;
  for (int k = 0; k < kRing && st == RR_OK; ++k) {
    if (hipHostMalloc(reinterpret_cast<void**>(&b->pinned[k]), b->desc_bytes, hipHostMallocDefault) != hipSuccess)
      st = RR_ERR_OUT_OF_MEMORY;
    else if (hipEventCreateWithFlags(&b->staged[k], hipEventDisableTiming) != hipSuccess)
      st = RR_ERR_DEVICE;
  }
  if (st == RR_OK && hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) st = RR_ERR_DEVICE;
  if (st != RR_OK) {
    (void)hipGetLastError();
    free_batch(b);
    return st;
  }
  *out = b;
  return RR_OK;
}

rr_status rr_batch_info(rr_batch b, int64_t* device_bytes, rr_batch_config* cfg) {
  if (!b) return RR_ERR_INVALID_ARGUMENT;
  if (device_bytes) *device_bytes = (int64_t)b->bytes;
  if (cfg) *cfg = b->cfg;
  return RR_OK;
}

rr_status rr_batch_set_config(rr_batch b, const rr_batch_config* cfg) {
  if (!b || !cfg || !valid_cfg(*cfg)) return RR_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(b->mu);
  b->cfg = *cfg;
  return RR_OK;
}

rr_status rr_batch_run(rr_batch b, const rr_segment* segs, int32_t nseg, uint32_t flags, void* stream) {
  if (!b) return RR_ERR_INVALID_ARGUMENT;
  if (flags & ~(RR_HITS_ORIGINAL_ORDER | RR_BATCH_EAGER)) return RR_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(b->mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device) return RR_ERR_INVALID_ARGUMENT;
  const int k = b->ring;
  if (b->staged_used[k] && hipEventSynchronize(b->staged[k]) != hipSuccess) return RR_ERR_DEVICE;
  uint32_t kb = 32;
  rr_status r = stage(b, segs, nseg, flags, b->cfg, b->pinned[k], &kb);
  if (r != RR_OK) return r;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(b->dev, b->pinned[k], b->desc_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return RR_ERR_DEVICE;
  if (hipEventRecord(b->staged[k], st) != hipSuccess) return RR_ERR_DEVICE;
  b->staged_used[k] = true;
  b->ring = (k + 1) % kRing;
  if (flags & RR_BATCH_EAGER) return enqueue(b, kb, b->cfg, st);
  hipGraphExec_t exec = nullptr;
  if ((r = graph_for(b, kb, b->cfg, &exec)) != RR_OK) return r;
  if (hipGraphLaunch(exec, st) != hipSuccess) return RR_ERR_DEVICE;
  return RR_OK;
}

rr_status rr_batch_autotune(rr_batch b, const rr_segment* segs, int32_t nseg, int32_t reps, rr_batch_config* best,
                            float* best_ms, void* stream) {
  if (!b || reps <= 0) return RR_ERR_INVALID_ARGUMENT;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return RR_ERR_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RR_ERR_DEVICE;
  }
  rr_batch_config keep;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    keep = b->cfg;
  }
  rr_batch_config win = keep;
  float win_ms = 1e30f;
  rr_status r = RR_OK;
  std::vector<rr_batch_config> shapes;
  for (uint32_t db : {8u, 4u})
    for (uint32_t kpt : {16u, 8u})
      for (uint32_t refill : {8u, 16u, 32u, 48u})
        for (uint32_t order : {RR_TILES_COUNTER, RR_TILES_FIXED})
          for (uint32_t block : {256u, 128u, 512u}) shapes.push_back({db, kpt, refill, order, block});
  for (const rr_batch_config& c : shapes) {
    if ((r = rr_batch_set_config(b, &c)) != RR_OK) break;
    if ((r = rr_batch_run(b, segs, nseg, 0, stream)) != RR_OK) break;  // capture + warm-up
    std::vector<float> t;
    for (int32_t i = 0; i < reps && r == RR_OK; ++i) {
      (void)hipEventRecord(e0, st);
      if ((r = rr_batch_run(b, segs, nseg, 0, stream)) != RR_OK) break;
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) {
        r = RR_ERR_DEVICE;
        break;
      }
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      t.push_back(ms);
    }
    if (r != RR_OK) break;
    std::sort(t.begin(), t.end());
    if (t[t.size() / 2] < win_ms) {
      win_ms = t[t.size() / 2];
      win = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)rr_batch_set_config(b, r == RR_OK ? &win : &keep);
  if (r != RR_OK) return r;
  if (best) *best = win;
  if (best_ms) *best_ms = win_ms;
  return RR_OK;
}

rr_status rr_batch_destroy(rr_batch b) {
  if (!b) return RR_ERR_INVALID_ARGUMENT;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  free_batch(b);
  (void)hipSetDevice(cur);
  return RR_OK;
}

}  // extern "C"
