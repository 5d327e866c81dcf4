// Internal declarations shared by the HIP translation units of librr.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "rr.h"

namespace rr {

// ------------------------------------------------------------- constants
constexpr int kWave = 64;              // gfx950 wavefront width
constexpr uint32_t kXcds = 8;          // MI355X: 8 accelerator dies (XCDs), 32 CUs each
constexpr int kMaxTreeDepth = 32;      // binary BVH leaf depth cap (the builder enforces it)
// A 4-wide traversal pushes at most 3 entries per level, and a 4-wide node is
// never deeper than the binary node it was collapsed from.
constexpr int kTraceStack4 = 3 * kMaxTreeDepth;
constexpr int32_t kEmptyChild = 0x7FFFFFFF;  // unused child slot of a 4-wide node
constexpr uint32_t kDefaultRefill = 16;      // idle lanes that trigger a wave refill (below 512 rays per wave)
constexpr uint32_t kStatusCountMask = 0x3FFFFFFFu;
constexpr uint32_t kStatusAggregate = 1u << 30;
constexpr uint32_t kStatusPrefix = 2u << 30;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// --------------------------------------------------------------- keys
// Per-component quantisation plan computed on the host from rr_key_params:
// component c (0-2 origin, 3-5 direction or termination point) owns
// bits[c] key slots, spaced `stride` apart, its least significant bit
// landing at key bit shift[c].
// One field of a general key layout: cnt bits of component comp, taken
// below its src_shift lowest bits, placed at key bits dst_shift,
// dst_shift + stride, ... (lowest first).
struct KeyField {
  uint8_t comp, cnt, stride, src_shift, dst_shift, pad[3];
};

constexpr int kMaxKeyFields = 12;
constexpr uint32_t kLengthCells = 1u << 20;

struct KeyPlan {
  float lo[3];
  float inv[3];
  float len;            // Two Point: fixed estimated length
  float scale[6];       // 2^bits as float
  uint32_t qmax[6];     // 2^bits - 1
  int32_t shift[6];
  int32_t kind;         // rr_key_kind
  int32_t key64;        // 0: 32-bit keys, 1: 64-bit keys
  // the figure's other layouts: components 0-2 origin, 3-5 direction (or
  // 3-4 octahedral u, v), placed field by field
  int32_t nfields;
  KeyField field[kMaxKeyFields];
  // Two Point Adaptive: the length table; Two Point Real: the rays' hits
  const void* aux;
  float E;              // largest box extent
  float s24;            // 2^24 / E: length-table units per unit length
};

rr_status make_key_plan(const rr_key_params* p, KeyPlan* out);

// Launchers (validated arguments; return RR_ERR_DEVICE on launch failure).
rr_status launch_keys(const rr_ray* rays, int64_t n, const uint8_t* alive, const KeyPlan& plan, void* keys,
                      uint32_t* idx, uint32_t* count_out, void* block_scratch, hipStream_t st);
rr_status launch_compact_only(int64_t n, const uint8_t* alive, uint32_t* idx, uint32_t* count_out,
                              void* block_scratch, hipStream_t st);
size_t keys_scratch_bytes(int64_t n);
// Two Point Adaptive length table (rr_length_cell[kLengthCells]).
rr_status launch_length_init(rr_length_cell* table, const KeyPlan& plan, float ratio, hipStream_t st);
// Adds hits[i] (i < min(*count_dev, n_max)) of rays[idx ? idx[i] : i].
rr_status launch_length_accumulate(rr_length_cell* table, const rr_ray* rays, const uint32_t* idx,
                                   const rr_hit* hits, int64_t n_max, const uint32_t* count_dev,
                                   const KeyPlan& plan, hipStream_t st);

// Capsule coherence measure of groups of 64 consecutive rays and its mean.
rr_status launch_coherence(const rr_ray* rays, const rr_hit* hits, int64_t n, float E, double* group_out,
                           double* mean_out, hipStream_t st);

// Block-wise sort of runs of `block` consecutive pairs (Section 3.2).
bool local_sort_supported(uint32_t key_bits, uint32_t block);
rr_status launch_local_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                            uint32_t block, hipStream_t st);

// --------------------------------------------------------------- sort
size_t sort_workspace_bytes(int64_t n_max, uint32_t key_bits, uint32_t digit_bits, uint32_t kpt);
// Keys of one sort tile for kpt keys per thread (the sort's block size times kpt).
uint32_t sort_tile_keys(uint32_t kpt);
// Keys per thread of rr_sort and the fused call for n keys: 8 (tiles of 4096
// keys) up to 2^24 keys, 16 (tiles of 8192, fewer tiles to look back over)
// beyond.
uint32_t sort_default_kpt(int64_t n);
size_t sort_workspace_bytes_any(int64_t n_max, uint32_t key_bits);
bool sort_config_supported(uint32_t key_bits, uint32_t digit_bits, uint32_t kpt);
// The LSD sort with an explicit digit width and tile size.
rr_status launch_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                      uint32_t digit_bits, uint32_t kpt, void* ws, size_t ws_bytes, hipStream_t st);
// rr_sort: the LSD sort with 8-bit digits; force_msd takes the
// most-significant-digit sort instead (64-bit keys below 2^27, else
// RR_ERR_UNSUPPORTED).
rr_status launch_sort_auto(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                           void* ws, size_t ws_bytes, hipStream_t st, bool force_msd = false);
// The same sort with the ray gather fused into its last pass:
// rays_out[i] = rays_in[idx[i]] for the sorted indices (n_max rays in); the
// keys are left unsorted.
rr_status launch_sort_gather(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                             uint32_t digit_bits, uint32_t kpt, void* ws, size_t ws_bytes, const rr_ray* rays_in,
                             rr_ray* rays_out, hipStream_t st, bool force_msd = false);

// ------------------------------------------------------ gather / scatter
rr_status launch_gather(const rr_ray* in, const uint32_t* idx, int64_t n_max, const uint32_t* count_dev, rr_ray* out,
                        hipStream_t st);
rr_status launch_scatter_hits(const rr_hit* in, const uint32_t* idx, int64_t n_max, const uint32_t* count_dev,
                              rr_hit* out, hipStream_t st);
rr_status launch_fill_miss(rr_hit* out, int64_t n, hipStream_t st);
rr_status launch_copy_u32(const uint32_t* in, uint32_t* out, int64_t n_max, const uint32_t* count_dev, hipStream_t st);
rr_status launch_iota(uint32_t* out, int64_t n, hipStream_t st);
rr_status launch_set_u32(uint32_t* out, uint32_t value, hipStream_t st);
rr_status launch_fill_u32(uint32_t* out, uint32_t n, uint32_t value, hipStream_t st);  // small n only

// --------------------------------------------------------------- scene
struct DeviceScene {
  float4* nodes = nullptr;   // 8 float4 per 4-wide inner node
  float4* tris = nullptr;    // 3 float4 per triangle, leaf order
  int32_t root = 0;          // inner node 0, or a leaf code
  int64_t n_nodes = 0;
  int64_t n_tris = 0;
  int32_t depth = 0;
  int32_t device = 0;
  int32_t quantised = 1;     // 64-byte nodes with 8-bit child bounds, else 128-byte nodes
  float lo[3], hi[3];
  size_t bytes = 0;
};

rr_status launch_trace_stats(const DeviceScene& s, const rr_ray* rays, int64_t n_max, rr_hit* hits,
                             uint64_t* stats_dev, hipStream_t st);
void trace_warm();
// block: threads per workgroup of the trace kernel, 128, 256 or 512.
rr_status launch_trace_refill(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                              const uint32_t* count_dev, rr_hit* hits, uint32_t refill, hipStream_t st,
                              uint32_t block = 256);
// Any-hit (occlusion) trace: some triangle hit in (tmin, tmax), or a miss.
rr_status launch_trace_any(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                           const uint32_t* count_dev, rr_hit* hits, hipStream_t st);
rr_status launch_trace(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                       const uint32_t* count_dev, rr_hit* hits, hipStream_t st);

// rr_reorder_and_trace with a workspace that is the library's static
// device array (scratch_bytes long, already known to be device memory).
rr_status reorder_and_trace_in_scratch(rr_scene_s* s, const rr_ray* rays, int64_t n, const uint8_t* alive,
                                       const rr_key_params* p, rr_hit* hits, uint32_t* perm_out,
                                       uint32_t* count_out, uint32_t flags, void* scratch, size_t scratch_bytes,
                                       void* stream);

}  // namespace rr

struct rr_scene_s {
  rr::DeviceScene d;
};

#define RR_LAUNCH_CHECK()                                   \
  do {                                                      \
    hipError_t e_ = hipGetLastError();                      \
    if (e_ != hipSuccess) return RR_ERR_DEVICE;             \
  } while (0)
