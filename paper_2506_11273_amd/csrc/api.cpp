// The C ABI of librr: argument validation, workspace layout and the
// composition of the kernels into the reordered trace.
#include <cmath>
#include <cstring>
#include <new>

#include "common.hpp"
#include "sort_seg.hpp"

namespace rr {
rr_status build_scene(const float* tris, int64_t n, int builder, DeviceScene* out);
}

using namespace rr;

namespace {

bool valid_n(int64_t n) { return n >= 0 && n < RR_MAX_RAYS; }

// Device pointers only: host memory passed where device memory is expected
// would fault inside a kernel, so it is rejected up front.
bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

struct ReorderLayout {
  size_t keys, idx, count, kscratch, sortws, rays, hits, total;
  size_t sort_bytes;
};

ReorderLayout reorder_layout(int64_t n, uint32_t key_bits) {
  ReorderLayout L{};
  size_t off = 0;
  const size_t kb = key_bits / 8;
  L.keys = off; off = align_up(off + kb * (size_t)n + 8, 256);
  L.idx = off; off = align_up(off + 4 * (size_t)n + 4, 256);
  L.count = off; off = align_up(off + 4, 256);
  L.kscratch = off; off = align_up(off + keys_scratch_bytes(n), 256);
  L.sort_bytes = sort_workspace_bytes_any(n, key_bits);
  L.sortws = off; off = align_up(off + L.sort_bytes, 256);
  L.rays = off; off = align_up(off + sizeof(rr_ray) * (size_t)n, 256);
  L.hits = off; off = align_up(off + sizeof(rr_hit) * (size_t)n, 256);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

const char* rr_status_string(rr_status s) {
  switch (s) {
    case RR_OK: return "ok";
    case RR_ERR_INVALID_ARGUMENT: return "invalid argument";
    case RR_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RR_ERR_DEVICE: return "device (HIP) error";
    case RR_ERR_UNSUPPORTED: return "unsupported";
    case RR_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case RR_ERR_BUDGET: return "over budget";
    default: return "unknown status";
  }
}

rr_status rr_device_count(int32_t* count) {
  if (!count) return RR_ERR_INVALID_ARGUMENT;
  int c = 0;
  if (hipGetDeviceCount(&c) != hipSuccess || c <= 0) {
    (void)hipGetLastError();
    *count = 0;
    return RR_ERR_DEVICE;
  }
  *count = c;
  return RR_OK;
}

// ------------------------------------------------------------------ scene

rr_status rr_scene_create_ex(const float* tri, int64_t n_tris, int32_t builder, rr_scene* out) {
  if (!out) return RR_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!tri || n_tris <= 0 || n_tris >= (int64_t(1) << 28)) return RR_ERR_INVALID_ARGUMENT;
  if ((builder & ~(1 | RR_BUILD_FULL_NODES)) != 0) return RR_ERR_INVALID_ARGUMENT;
  // finite coordinates below 1e18 in magnitude keep every traversal term finite
  for (int64_t i = 0; i < 9 * n_tris; ++i)
    if (!(std::fabs(tri[i]) < 1e18f)) return RR_ERR_INVALID_ARGUMENT;
  rr_scene s = new (std::nothrow) rr_scene_s;
  if (!s) return RR_ERR_OUT_OF_MEMORY;
  rr_status st;
  try {
    st = build_scene(tri, n_tris, builder, &s->d);
  } catch (const std::bad_alloc&) {
    st = RR_ERR_OUT_OF_MEMORY;
  } catch (...) {
    st = RR_ERR_DEVICE;
  }
  if (st != RR_OK) {
    delete s;
    return st;
  }
  *out = s;
  return RR_OK;
}

rr_status rr_scene_create(const float* tri, int64_t n_tris, rr_scene* out) {
  return rr_scene_create_ex(tri, n_tris, 1, out);
}

rr_status rr_scene_bounds(rr_scene s, float lo[3], float hi[3]) {
  if (!s || !lo || !hi) return RR_ERR_INVALID_ARGUMENT;
  for (int k = 0; k < 3; ++k) {
    lo[k] = s->d.lo[k];
    hi[k] = s->d.hi[k];
  }
  return RR_OK;
}

rr_status rr_scene_info(rr_scene s, int64_t* nodes, int32_t* depth, int64_t* device_bytes) {
  if (!s) return RR_ERR_INVALID_ARGUMENT;
  if (nodes) *nodes = s->d.n_nodes;
  if (depth) *depth = s->d.depth;
  if (device_bytes) *device_bytes = (int64_t)s->d.bytes;
  return RR_OK;
}

rr_status rr_scene_destroy(rr_scene s) {
  if (!s) return RR_ERR_INVALID_ARGUMENT;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(s->d.device);
  (void)hipFree(s->d.nodes);
  (void)hipFree(s->d.tris);
  (void)hipSetDevice(cur);
  delete s;
  return RR_OK;
}

// ------------------------------------------------------------------- keys

rr_status rr_keys_workspace_size(int64_t n, size_t* bytes) {
  if (!bytes || !valid_n(n)) return RR_ERR_INVALID_ARGUMENT;
  *bytes = keys_scratch_bytes(n);
  return RR_OK;
}

rr_status rr_compute_keys(const rr_ray* rays, int64_t n, const uint8_t* alive, const rr_key_params* p,
                          void* keys_out, uint32_t* idx_out, uint32_t* count_out, void* workspace, size_t ws_bytes,
                          void* stream) {
  if (!valid_n(n) || !p) return RR_ERR_INVALID_ARGUMENT;
  KeyPlan plan;
  rr_status st = make_key_plan(p, &plan);
  if (st != RR_OK) return st;
  if (plan.aux && (!is_device_ptr(plan.aux) || !aligned(plan.aux, 16))) return RR_ERR_INVALID_ARGUMENT;
  if (alive && !count_out) return RR_ERR_INVALID_ARGUMENT;
  if (count_out && !is_device_ptr(count_out)) return RR_ERR_INVALID_ARGUMENT;
  if (n == 0) return count_out ? launch_set_u32(count_out, 0u, S(stream)) : RR_OK;
  if (!is_device_ptr(rays) || !aligned(rays, 16) || !is_device_ptr(keys_out) || !is_device_ptr(idx_out))
    return RR_ERR_INVALID_ARGUMENT;
  if (!aligned(keys_out, p->key_bits / 8) || !aligned(idx_out, 4)) return RR_ERR_INVALID_ARGUMENT;
  if (alive) {
    if (!is_device_ptr(alive)) return RR_ERR_INVALID_ARGUMENT;
    if (!workspace || !is_device_ptr(workspace)) return RR_ERR_INVALID_ARGUMENT;
    if (ws_bytes < keys_scratch_bytes(n)) return RR_ERR_WORKSPACE_TOO_SMALL;
  }
  return launch_keys(rays, n, alive, plan, keys_out, idx_out, count_out, workspace, S(stream));
}

// ----------------------------------------------------------- length table

rr_status rr_length_table_init(rr_length_cell* table, const rr_key_params* p, void* stream) {
  if (!table || !p) return RR_ERR_INVALID_ARGUMENT;
  if (!is_device_ptr(table) || !aligned(table, 16)) return RR_ERR_INVALID_ARGUMENT;
  if (!(p->term_ratio >= 0.0f)) return RR_ERR_INVALID_ARGUMENT;
  rr_key_params q = *p;
  q.kind = RR_KEY_ORIGIN_TERMINATION;
  q.key_bits = 32;
  KeyPlan plan;
  rr_status st = make_key_plan(&q, &plan);
  if (st != RR_OK) return st;
  return launch_length_init(table, plan, p->term_ratio, S(stream));
}

rr_status rr_length_table_accumulate(rr_length_cell* table, const rr_ray* rays, const uint32_t* idx,
                                     const rr_hit* hits, int64_t n, const uint32_t* count_dev,
                                     const rr_key_params* p, void* stream) {
  if (!table || !p || !valid_n(n)) return RR_ERR_INVALID_ARGUMENT;
  if (n == 0) return RR_OK;
  if (!is_device_ptr(table) || !aligned(table, 16) || !is_device_ptr(rays) || !aligned(rays, 16) ||
      !is_device_ptr(hits) || !aligned(hits, 16))
    return RR_ERR_INVALID_ARGUMENT;
  if ((idx && (!is_device_ptr(idx) || !aligned(idx, 4))) || (count_dev && !is_device_ptr(count_dev)))
    return RR_ERR_INVALID_ARGUMENT;
  rr_key_params q = *p;
  q.kind = RR_KEY_ORIGIN_TERMINATION;
  q.key_bits = 32;
  KeyPlan plan;
  rr_status st = make_key_plan(&q, &plan);
  if (st != RR_OK) return st;
  return launch_length_accumulate(table, rays, idx, hits, n, count_dev, plan, S(stream));
}

// -------------------------------------------------------------- coherence

rr_status rr_coherence_m64(const rr_ray* rays, const rr_hit* hits, int64_t n, const rr_key_params* p,
                           double* group_out, double* mean_out, void* stream) {
  if (!p || !valid_n(n) || !mean_out || !is_device_ptr(mean_out) || !aligned(mean_out, 8))
    return RR_ERR_INVALID_ARGUMENT;
  if (n > 0 && (!is_device_ptr(rays) || !aligned(rays, 16) || !is_device_ptr(hits) || !aligned(hits, 16) ||
                !group_out || !is_device_ptr(group_out) || !aligned(group_out, 8)))
    return RR_ERR_INVALID_ARGUMENT;
  float E = p->box_hi[0] - p->box_lo[0];
  for (int k = 1; k < 3; ++k)
    if (p->box_hi[k] - p->box_lo[k] > E) E = p->box_hi[k] - p->box_lo[k];
  return launch_coherence(rays, hits, n, E, group_out, mean_out, S(stream));
}

// ------------------------------------------------------------------- sort

rr_status rr_sort_workspace_size(int64_t n_max, uint32_t key_bits, size_t* bytes) {
  if (!bytes || !valid_n(n_max) || (key_bits != 32 && key_bits != 64)) return RR_ERR_INVALID_ARGUMENT;
  *bytes = sort_workspace_bytes_any(n_max, key_bits);
  return RR_OK;
}

rr_status rr_sort_ex(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                     uint32_t digit_bits, uint32_t kpt, void* workspace, size_t ws_bytes, void* stream) {
  if (!valid_n(n_max) || (key_bits != 32 && key_bits != 64)) return RR_ERR_INVALID_ARGUMENT;
  if (!sort_config_supported(key_bits, digit_bits, kpt)) return RR_ERR_UNSUPPORTED;
  if (n_max == 0) return RR_OK;
  if (!is_device_ptr(keys) || !is_device_ptr(idx) || !is_device_ptr(workspace)) return RR_ERR_INVALID_ARGUMENT;
  if (!aligned(keys, key_bits / 8) || !aligned(idx, 4) || !aligned(workspace, 256)) return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  if (ws_bytes < sort_workspace_bytes(n_max, key_bits, digit_bits, kpt)) return RR_ERR_WORKSPACE_TOO_SMALL;
  return launch_sort(keys, idx, n_max, count_dev, key_bits, digit_bits, kpt, workspace, ws_bytes, S(stream));
}

rr_status rr_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                  void* workspace, size_t ws_bytes, void* stream) {
  if (!valid_n(n_max) || (key_bits != 32 && key_bits != 64)) return RR_ERR_INVALID_ARGUMENT;
  if (n_max == 0) return RR_OK;
  if (!is_device_ptr(keys) || !is_device_ptr(idx) || !is_device_ptr(workspace)) return RR_ERR_INVALID_ARGUMENT;
  if (!aligned(keys, key_bits / 8) || !aligned(idx, 4) || !aligned(workspace, 256)) return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  if (ws_bytes < sort_workspace_bytes_any(n_max, key_bits)) return RR_ERR_WORKSPACE_TOO_SMALL;
  return launch_sort_auto(keys, idx, n_max, count_dev, key_bits, workspace, ws_bytes, S(stream));
}

rr_status rr_sort_msd(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                      void* workspace, size_t ws_bytes, void* stream) {
  if (!valid_n(n_max) || (key_bits != 32 && key_bits != 64)) return RR_ERR_INVALID_ARGUMENT;
  if (n_max == 0) return RR_OK;
  if (!msd_supported(n_max, key_bits)) return RR_ERR_UNSUPPORTED;
  if (!is_device_ptr(keys) || !is_device_ptr(idx) || !is_device_ptr(workspace)) return RR_ERR_INVALID_ARGUMENT;
  if (!aligned(keys, key_bits / 8) || !aligned(idx, 4) || !aligned(workspace, 256)) return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  if (ws_bytes < sort_workspace_bytes_any(n_max, key_bits)) return RR_ERR_WORKSPACE_TOO_SMALL;
  return launch_sort_auto(keys, idx, n_max, count_dev, key_bits, workspace, ws_bytes, S(stream), true);
}

rr_status rr_local_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                        uint32_t block, void* stream) {
  if (!valid_n(n_max) || (key_bits != 32 && key_bits != 64)) return RR_ERR_INVALID_ARGUMENT;
  if (!local_sort_supported(key_bits, block)) return RR_ERR_UNSUPPORTED;
  if (n_max == 0) return RR_OK;
  if (!is_device_ptr(keys) || !is_device_ptr(idx) || !aligned(keys, key_bits / 8) || !aligned(idx, 4))
    return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  return launch_local_sort(keys, idx, n_max, count_dev, key_bits, block, S(stream));
}

// ----------------------------------------------------------------- gather

rr_status rr_gather(const rr_ray* in, const uint32_t* idx, int64_t n_max, const uint32_t* count_dev, rr_ray* out,
                    void* stream) {
  if (!valid_n(n_max)) return RR_ERR_INVALID_ARGUMENT;
  if (n_max == 0) return RR_OK;
  if (!is_device_ptr(in) || !is_device_ptr(idx) || !is_device_ptr(out)) return RR_ERR_INVALID_ARGUMENT;
  if (!aligned(in, 16) || !aligned(out, 16) || !aligned(idx, 4)) return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  const char* a = reinterpret_cast<const char*>(in);
  const char* b = reinterpret_cast<const char*>(out);
  const size_t bytes = sizeof(rr_ray) * (size_t)n_max;
  if (a < b + bytes && b < a + bytes) return RR_ERR_INVALID_ARGUMENT;
  return launch_gather(in, idx, n_max, count_dev, out, S(stream));
}

rr_status rr_scatter_hits(const rr_hit* in, const uint32_t* idx, int64_t n_max, const uint32_t* count_dev,
                          rr_hit* out, void* stream) {
  if (!valid_n(n_max)) return RR_ERR_INVALID_ARGUMENT;
  if (n_max == 0) return RR_OK;
  if (!is_device_ptr(in) || !is_device_ptr(idx) || !is_device_ptr(out)) return RR_ERR_INVALID_ARGUMENT;
  if (!aligned(in, 16) || !aligned(out, 16) || !aligned(idx, 4)) return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  const char* a = reinterpret_cast<const char*>(in);
  const char* b = reinterpret_cast<const char*>(out);
  const size_t bytes = sizeof(rr_hit) * (size_t)n_max;
  if (a < b + bytes && b < a + bytes) return RR_ERR_INVALID_ARGUMENT;
  return launch_scatter_hits(in, idx, n_max, count_dev, out, S(stream));
}

// ------------------------------------------------------------------ trace

rr_status rr_trace(rr_scene s, const rr_ray* rays, int64_t n_max, const uint32_t* count_dev, rr_hit* hits,
                   void* stream) {
  if (!s || !valid_n(n_max)) return RR_ERR_INVALID_ARGUMENT;
  if (n_max == 0) return RR_OK;
  if (!is_device_ptr(rays) || !is_device_ptr(hits) || !aligned(rays, 16) || !aligned(hits, 16))
    return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->d.device) return RR_ERR_INVALID_ARGUMENT;
  return launch_trace(s->d, rays, nullptr, n_max, count_dev, hits, S(stream));
}

rr_status rr_trace_any(rr_scene s, const rr_ray* rays, int64_t n_max, const uint32_t* count_dev, rr_hit* hits,
                       void* stream) {
  if (!s || !valid_n(n_max)) return RR_ERR_INVALID_ARGUMENT;
  if (n_max == 0) return RR_OK;
  if (!is_device_ptr(rays) || !is_device_ptr(hits) || !aligned(rays, 16) || !aligned(hits, 16))
    return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->d.device) return RR_ERR_INVALID_ARGUMENT;
  return launch_trace_any(s->d, rays, nullptr, n_max, count_dev, hits, S(stream));
}

rr_status rr_trace_ex(rr_scene s, const rr_ray* rays, int64_t n_max, const uint32_t* count_dev, rr_hit* hits,
                      uint32_t refill, void* stream) {
  if (!s || !valid_n(n_max) || refill < 1 || refill > 64) return RR_ERR_INVALID_ARGUMENT;
  if (n_max == 0) return RR_OK;
  if (!is_device_ptr(rays) || !is_device_ptr(hits) || !aligned(rays, 16) || !aligned(hits, 16))
    return RR_ERR_INVALID_ARGUMENT;
  if (count_dev && !is_device_ptr(count_dev)) return RR_ERR_INVALID_ARGUMENT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->d.device) return RR_ERR_INVALID_ARGUMENT;
  return launch_trace_refill(s->d, rays, nullptr, n_max, count_dev, hits, refill, S(stream));
}

rr_status rr_trace_profile(rr_scene s, const rr_ray* rays, int64_t n, rr_hit* hits, uint64_t* stats_dev,
                           void* stream) {
  if (!s || !valid_n(n)) return RR_ERR_INVALID_ARGUMENT;
  if (!is_device_ptr(stats_dev) || !aligned(stats_dev, 8)) return RR_ERR_INVALID_ARGUMENT;
  rr_status r = launch_fill_u32(reinterpret_cast<uint32_t*>(stats_dev), 2 * RR_TRACE_PROFILE_COUNTERS, 0u, S(stream));
  if (r != RR_OK || n == 0) return r;
  if (!is_device_ptr(rays) || !is_device_ptr(hits) || !aligned(rays, 16) || !aligned(hits, 16))
    return RR_ERR_INVALID_ARGUMENT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->d.device) return RR_ERR_INVALID_ARGUMENT;
  return launch_trace_stats(s->d, rays, n, hits, stats_dev, S(stream));
}

// --------------------------------------------------------- fused pipeline

rr_status rr_reorder_workspace_size(int64_t n_max, const rr_key_params* p, size_t* bytes) {
  if (!bytes || !p || !valid_n(n_max)) return RR_ERR_INVALID_ARGUMENT;
  const uint32_t kb = p->kind == RR_KEY_NONE ? 32u : p->key_bits;
  if (kb != 32 && kb != 64) return RR_ERR_INVALID_ARGUMENT;
  *bytes = reorder_layout(n_max, kb).total;
  return RR_OK;
}

}  // extern "C"

namespace {

// rr_reorder_and_trace; ws_is_scratch: the workspace is the library's own
// static device array (its size checked by the caller), not caller memory.
rr_status reorder_and_trace(rr_scene s, const rr_ray* rays, int64_t n, const uint8_t* alive,
                            const rr_key_params* p, rr_hit* hits, uint32_t* perm_out, uint32_t* count_out,
                            uint32_t flags, void* workspace, size_t ws_bytes, void* stream, bool ws_is_scratch) {
  if (!s || !p || !valid_n(n)) return RR_ERR_INVALID_ARGUMENT;
  constexpr uint32_t kLocal = RR_LOCAL_SORT_1024 | RR_LOCAL_SORT_2048 | RR_LOCAL_SORT_4096;
  if (flags & ~(RR_HITS_ORIGINAL_ORDER | RR_INDIRECT | RR_ANY_HIT | RR_SORT_MSD | kLocal))
    return RR_ERR_INVALID_ARGUMENT;
  const bool any = (flags & RR_ANY_HIT) != 0;
  const uint32_t local = flags & kLocal;
  if (local & (local - 1)) return RR_ERR_INVALID_ARGUMENT;  // at most one block size
  const uint32_t local_block = local == RR_LOCAL_SORT_1024 ? 1024u
                               : local == RR_LOCAL_SORT_2048 ? 2048u
                               : local == RR_LOCAL_SORT_4096 ? 4096u
                                                             : 0u;
  const bool sorted = p->kind != RR_KEY_NONE;
  const bool force_msd = sorted && (flags & RR_SORT_MSD) != 0;
  if (force_msd && local_block) return RR_ERR_INVALID_ARGUMENT;
  KeyPlan plan{};
  if (sorted) {
    rr_status st = make_key_plan(p, &plan);
    if (st != RR_OK) return st;
    if (plan.aux && (!is_device_ptr(plan.aux) || !aligned(plan.aux, 16))) return RR_ERR_INVALID_ARGUMENT;
    if (any && plan.kind == RR_KEY_TWO_POINT_ADAPTIVE) return RR_ERR_INVALID_ARGUMENT;
  }
  hipStream_t st = S(stream);
  if (count_out && !is_device_ptr(count_out)) return RR_ERR_INVALID_ARGUMENT;
  if (n == 0) return count_out ? launch_set_u32(count_out, 0u, st) : RR_OK;
  if (!is_device_ptr(rays) || !is_device_ptr(hits) || !aligned(rays, 16) || !aligned(hits, 16))
    return RR_ERR_INVALID_ARGUMENT;
  if (alive && !is_device_ptr(alive)) return RR_ERR_INVALID_ARGUMENT;
  if (perm_out && (!is_device_ptr(perm_out) || !aligned(perm_out, 4))) return RR_ERR_INVALID_ARGUMENT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->d.device) return RR_ERR_INVALID_ARGUMENT;
  const uint32_t kb = sorted ? p->key_bits : 32u;
  if (force_msd && !msd_supported(n, kb)) return RR_ERR_UNSUPPORTED;
  const ReorderLayout L = reorder_layout(n, kb);
  if (!workspace || (!ws_is_scratch && !is_device_ptr(workspace)) || !aligned(workspace, 256))
    return RR_ERR_INVALID_ARGUMENT;
  if (ws_bytes < L.total) return RR_ERR_WORKSPACE_TOO_SMALL;

  char* w = reinterpret_cast<char*>(workspace);
  void* keys = w + L.keys;
  uint32_t* idx = reinterpret_cast<uint32_t*>(w + L.idx);
  uint32_t* cnt = alive ? reinterpret_cast<uint32_t*>(w + L.count) : nullptr;
  rr_ray* srays = reinterpret_cast<rr_ray*>(w + L.rays);
  rr_hit* shits = reinterpret_cast<rr_hit*>(w + L.hits);
  const bool orig = (flags & RR_HITS_ORIGINAL_ORDER) != 0;
  const bool indirect = (flags & RR_INDIRECT) != 0;
  rr_status r;

  if (!sorted && !alive) {
    // identity order: trace in place, both hit orders coincide
    r = any ? launch_trace_any(s->d, rays, nullptr, n, nullptr, hits, st)
            : launch_trace(s->d, rays, nullptr, n, nullptr, hits, st);
    if (r != RR_OK) return r;
    if (perm_out && (r = launch_iota(perm_out, n, st)) != RR_OK) return r;
    if (count_out && (r = launch_set_u32(count_out, (uint32_t)n, st)) != RR_OK) return r;
    return RR_OK;
  }

  bool gathered = false;  // srays already hold the rays in key order
  if (sorted && !alive && !local_block && !indirect) {
    // dense device-wide sort: the keys kernel also counts the digits, and
    // the sort's last pass gathers the rays
    if ((r = launch_keys_sort_gather(rays, n, plan, keys, idx, sort_default_kpt(n), w + L.sortws, L.sort_bytes, srays,
                                     st, force_msd)) != RR_OK)
      return r;
    gathered = true;
  } else if (sorted) {
    if ((r = launch_keys(rays, n, alive, plan, keys, idx, cnt, w + L.kscratch, st)) != RR_OK) return r;
    if (local_block) {
      if ((r = launch_local_sort(keys, idx, n, cnt, kb, local_block, st)) != RR_OK) return r;
    } else if (!indirect) {
      // the device-wide sort's last pass also gathers the rays
      if ((r = launch_sort_gather(keys, idx, n, cnt, kb, 8, sort_default_kpt(n), w + L.sortws, L.sort_bytes, rays, srays,
                                  st, force_msd)) != RR_OK)
        return r;
      gathered = true;
    } else if ((r = launch_sort_auto(keys, idx, n, cnt, kb, w + L.sortws, L.sort_bytes, st, force_msd)) != RR_OK) {
      return r;
    }
  } else {
    if ((r = launch_compact_only(n, alive, idx, cnt, w + L.kscratch, st)) != RR_OK) return r;
  }
  rr_hit* tout = orig ? shits : hits;
  auto trace = any ? launch_trace_any : launch_trace;
  if (indirect) {
    if ((r = trace(s->d, rays, idx, n, cnt, tout, st)) != RR_OK) return r;
  } else {
    if (!gathered && (r = launch_gather(rays, idx, n, cnt, srays, st)) != RR_OK) return r;
    if ((r = trace(s->d, srays, nullptr, n, cnt, tout, st)) != RR_OK) return r;
  }
  if (plan.kind == RR_KEY_TWO_POINT_ADAPTIVE) {
    // Section 3.1.6: the traced lengths update the table after each trace
    rr_length_cell* table = const_cast<rr_length_cell*>(reinterpret_cast<const rr_length_cell*>(plan.aux));
    if ((r = launch_length_accumulate(table, rays, idx, tout, n, cnt, plan, st)) != RR_OK) return r;
  }
  if (orig) {
    if (alive && (r = launch_fill_miss(hits, n, st)) != RR_OK) return r;
    if ((r = launch_scatter_hits(shits, idx, n, cnt, hits, st)) != RR_OK) return r;
  }
  if (perm_out && (r = launch_copy_u32(idx, perm_out, n, cnt, st)) != RR_OK) return r;
  if (count_out) {
    if (cnt) {
      if ((r = launch_copy_u32(cnt, count_out, 1, nullptr, st)) != RR_OK) return r;
    } else if ((r = launch_set_u32(count_out, (uint32_t)n, st)) != RR_OK) {
      return r;
    }
  }
  return RR_OK;
}

}  // namespace

namespace rr {

rr_status reorder_and_trace_in_scratch(rr_scene s, const rr_ray* rays, int64_t n, const uint8_t* alive,
                                       const rr_key_params* p, rr_hit* hits, uint32_t* perm_out,
                                       uint32_t* count_out, uint32_t flags, void* scratch, size_t scratch_bytes,
                                       void* stream) {
  return reorder_and_trace(s, rays, n, alive, p, hits, perm_out, count_out, flags, scratch, scratch_bytes, stream,
                           true);
}

}  // namespace rr

extern "C" {

rr_status rr_reorder_and_trace(rr_scene s, const rr_ray* rays, int64_t n, const uint8_t* alive,
                               const rr_key_params* p, rr_hit* hits, uint32_t* perm_out, uint32_t* count_out,
                               uint32_t flags, void* workspace, size_t ws_bytes, void* stream) {
  return reorder_and_trace(s, rays, n, alive, p, hits, perm_out, count_out, flags, workspace, ws_bytes, stream,
                           false);
}

}  // extern "C"
