/*
 * rr.h -- ray reordering and closest-hit tracing on AMD Instinct MI355X (gfx950).
 *
 * Implements the data-parallel path of Meister, Boksansky, Guthe and Bittner,
 * "On Ray Reordering Techniques for Faster GPU Ray Tracing" (I3D 2020):
 * per-ray sort keys (Section 3.1, Figure "codes"), a key/index sort
 * (Section 3.2), the ray-data reordering pass (Section 3.2, Section 4.4.1)
 * and the closest-hit trace the reordering is meant to speed up (Section 4.1).
 *
 * Conventions for every function below:
 *  - All functions are extern "C", never throw, and return rr_status.
 *  - Array arguments are DEVICE pointers owned by the caller unless stated
 *    otherwise; the library never frees them.  Sizes are element counts.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *    the default stream).  No function waits for the device unless stated.
 *  - Argument errors are detected on the host before anything is enqueued
 *    and return RR_ERR_INVALID_ARGUMENT (or RR_ERR_WORKSPACE_TOO_SMALL /
 *    RR_ERR_UNSUPPORTED); launch failures return RR_ERR_DEVICE.  Faults
 *    inside kernels surface at the caller's next synchronisation.
 *  - n = 0 is valid and enqueues nothing (except that count outputs are
 *    written as 0).
 *  - Buffers given to one call must not overlap unless stated otherwise.
 *  - The functions of this header allocate device memory only in
 *    rr_scene_create (owned by the scene, freed by rr_scene_destroy);
 *    rr_batch_create and rr_server_create (rr_batch.h) allocate the buffers
 *    of a batch.  Everything else works in caller-provided memory.
 */
#ifndef RR_H
#define RR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rr_status;
#define RR_OK 0
#define RR_ERR_INVALID_ARGUMENT (-1)
#define RR_ERR_OUT_OF_MEMORY (-2)
#define RR_ERR_DEVICE (-3)
#define RR_ERR_UNSUPPORTED (-4)
#define RR_ERR_WORKSPACE_TOO_SMALL (-5)
#define RR_ERR_BUDGET (-6)

/* Bound on the ray count of a single call: calls accept n < RR_MAX_RAYS, so
 * at most 2^30 - 1 rays (the sort's tile status words hold 30-bit counts). */
#define RR_MAX_RAYS ((int64_t)1 << 30)

/* A ray (Section 3: origin, direction and extent), 32 bytes, 16-byte
 * aligned.  Valid hits satisfy tmin < t < tmax.  Directions are expected to
 * be unit length (the keys quantise each component over [-1, 1]). */
typedef struct rr_ray {
  float org[3];
  float tmin;
  float dir[3];
  float tmax;
} rr_ray;

/* Closest hit, 16 bytes.  prim is the index of the triangle in the array
 * given to rr_scene_create; (u, v) are its barycentric coordinates along
 * (v1 - v0, v2 - v0).  A miss is {+inf, -1, 0, 0}. */
typedef struct rr_hit {
  float t;
  int32_t prim;
  float u, v;
} rr_hit;

/* Sort-key methods of Section 3.1 and Figure "codes". */
typedef enum rr_key_kind {
  RR_KEY_NONE = 0,                 /* no reordering (identity order) */
  RR_KEY_ORIGIN_DIRECTION = 1,     /* Section 3.1.2 (Reis et al.): origin bits above direction bits */
  RR_KEY_ORIGIN_TERMINATION = 2,   /* Section 3.1.5 "Two Point": origin and estimated termination
                                      point interleaved, fixed-length estimate of Section 3.1.6 */
  RR_KEY_ORIGIN = 3,               /* Section 3.1.1: origin only */
  RR_KEY_DIRECTION_ORIGIN = 4,     /* Section 3.1.3 (Costa et al.): direction bits above origin bits */
  RR_KEY_AILA = 5,                 /* Section 3.1.4 (Aila and Karras): origin and direction
                                      interleaved, three leading zero bits per direction component */
  RR_KEY_AILA_COMPACT = 6,         /* Section 3.1.4: the compacted variant, no zero bits */
  RR_KEY_OCTAHEDRON = 7,           /* Section 3.1.4: origin with an octahedral direction */
  RR_KEY_TWO_POINT_ADAPTIVE = 8,   /* Section 3.1.6: Two Point, length from a length table */
  RR_KEY_TWO_POINT_REAL = 9        /* Section 3.1.6 reference: Two Point at the traced termination */
} rr_key_kind;

/* Key parameters.
 *  kind        one of rr_key_kind.
 *  key_bits    32 or 64; kinds 3-7 exist with 32 bits only (the layouts of
 *              Figure "codes"); RR_ERR_UNSUPPORTED otherwise.
 *  box_lo/hi   quantisation box for origins and termination points, normally
 *              the scene bounds (rr_scene_bounds).  A flat axis quantises to 0.
 *  term_ratio  Two Point kinds: the fixed estimated ray length is term_ratio
 *              x the largest box extent E, capped at the ray's tmax (Section
 *              3.1.6 uses 0.25); it is also the length of the dummy ray each
 *              length-table cell starts with.
 *  origin_bits origin-direction only: number of origin bits; 0 selects 22
 *              for 32-bit keys (Figure "codes", Reis row) and 44 for 64-bit.
 *  aux         RR_KEY_TWO_POINT_ADAPTIVE: the device length table
 *              (rr_length_cell[RR_LENGTH_CELLS], see rr_length_table_init);
 *              RR_KEY_TWO_POINT_REAL: device rr_hit[n], hits[i] the traced hit
 *              of rays[i]; NULL (ignored) for the other kinds.
 * Bit layouts, most significant first; a run cycles the components x, y, z
 * (u, v for the octahedral direction):
 *   origin-direction  origin_bits slots of o, then key_bits - origin_bits of d
 *   Two Point (2/8/9) key_bits slots cycling (o.x, o.y, o.z, t.x, t.y, t.z)
 *   origin            o32
 *   direction-origin  d8 o24
 *   Aila              (o3 d3) x 5, o2, the first three slots of each direction
 *                     component are zero bits
 *   Aila Compact      o12 d3 o3 d3 o3 d3 o3 d2
 *   octahedron        o15 q2 o3 q2 o3 q2 o3 q2, q the octahedral (u, v)
 * A component owning b slots is quantised as
 * q = min(trunc(clamp((x - lo) / (hi - lo), 0, 1) * 2^b), 2^b - 1)
 * (directions and octahedral coordinates use lo = -1, hi = 1), its most
 * significant bit in its first slot.  The octahedral coordinates of d are
 * (x, y) of d / (|d.x| + |d.y| + |d.z|), folded for d.z < 0 to
 * ((1 - |y|) sgn x, (1 - |x|) sgn y) with sgn(0) = +1.  Two Point Real uses
 * the traced length for hits and the fixed estimate for misses. */
typedef struct rr_key_params {
  int32_t kind;
  uint32_t key_bits;
  float box_lo[3];
  float box_hi[3];
  float term_ratio;
  uint32_t origin_bits;
  const void* aux;
} rr_key_params;

/* Two Point Adaptive length table (Section 3.1.6): RR_LENGTH_CELLS cells
 * indexed by the 20-bit Aila Compact code of a ray (the 20 leading slots of
 * that layout: origin 5/5/5 bits, direction 2/2/1 bits), each holding the sum
 * of the lengths of the rays traced from it and their count.  Lengths are
 * held in units of E / 2^24 (E the largest box extent) and truncated, so
 * sums do not depend on the order rays are added in; the estimate is
 * (float)(sum * E / (count * 2^24)) in double precision. */
#define RR_LENGTH_CELLS (1u << 20)
typedef struct rr_length_cell {
  uint64_t sum;
  uint32_t count;
  uint32_t unused;
} rr_length_cell;

typedef struct rr_scene_s* rr_scene;

const char* rr_status_string(rr_status s);

/* Number of visible HIP devices; fails with RR_ERR_DEVICE when none. */
rr_status rr_device_count(int32_t* count);

/* ------------------------------------------------------------------ scene
 * Builds a BVH over n_tris triangles and uploads it to the current
 * device.  tri_xyz_host is a HOST array of n_tris x 9 floats
 * {v0.xyz, v1.xyz, v2.xyz}, read during the call only; coordinates must be
 * finite and below 1e18 in magnitude (RR_ERR_INVALID_ARGUMENT otherwise).  The scene owns its
 * device memory until rr_scene_destroy; it is immutable and may be shared
 * by concurrent calls on any stream of that device.
 *  builder (rr_scene_create_ex): 0 = median split (balanced), 1 = binned
 *  surface area heuristic (what rr_scene_create uses); or'ed with
 *  RR_BUILD_FULL_NODES, the 4-wide nodes keep full binary32 child bounds
 *  (128 bytes) instead of 8-bit bounds quantised outward against the parent
 *  box (64 bytes).  Results of rr_trace do not depend on either choice. */
#define RR_BUILD_FULL_NODES 2
rr_status rr_scene_create(const float* tri_xyz_host, int64_t n_tris, rr_scene* out);
rr_status rr_scene_create_ex(const float* tri_xyz_host, int64_t n_tris, int32_t builder, rr_scene* out);
rr_status rr_scene_bounds(rr_scene s, float lo[3], float hi[3]);
/* Node count, tree depth and device bytes of the scene (any pointer may be NULL). */
rr_status rr_scene_info(rr_scene s, int64_t* nodes, int32_t* depth, int64_t* device_bytes);
rr_status rr_scene_destroy(rr_scene s);

/* ------------------------------------------------------------------- keys
 * Section 3.1: one key per ray.  keys_out holds uint32 (key_bits 32) or
 * uint64 (key_bits 64) values; idx_out receives the ray index of each key.
 * Without `alive` (NULL): keys_out[i] is the key of rays[i] and idx_out[i] = i;
 * workspace may be NULL.
 * With `alive` (n bytes, non-zero = live): only live rays are kept, in
 * ascending index order (stable compaction of the terminated slots), and
 * *count_out (device uint32, required) receives their number; entries past
 * the count are left untouched.  The compaction needs a device workspace of
 * rr_keys_workspace_size bytes (overwritten).  When alive is NULL, count_out
 * may be NULL, else n is written to it.  kind must not be RR_KEY_NONE. */
rr_status rr_keys_workspace_size(int64_t n, size_t* bytes);
rr_status rr_compute_keys(const rr_ray* rays, int64_t n, const uint8_t* alive, const rr_key_params* p,
                          void* keys_out, uint32_t* idx_out, uint32_t* count_out, void* workspace, size_t ws_bytes,
                          void* stream);

/* Length table of Two Point Adaptive (Section 3.1.6).
 * rr_length_table_init writes every cell of the device table (RR_LENGTH_CELLS
 * x 16 bytes, caller-owned) as one dummy ray of length p->term_ratio x E:
 * {trunc(term_ratio * 2^24), 1}.  rr_length_table_accumulate adds the traced
 * length of every hit (prim >= 0) among hits[0, n) to the cell of the ray
 * it belongs to, rays[idx ? idx[i] : i] for hits[i]; with count_dev (device
 * uint32) only the first min(*count_dev, n) hits.  Adding is atomic and
 * exact, so concurrent calls on one table commute.  p gives the
 * quantisation box (its kind is not used).  rr_reorder_and_trace with
 * RR_KEY_TWO_POINT_ADAPTIVE calls it for the rays it traced. */
rr_status rr_length_table_init(rr_length_cell* table, const rr_key_params* p, void* stream);
rr_status rr_length_table_accumulate(rr_length_cell* table, const rr_ray* rays, const uint32_t* idx,
                                     const rr_hit* hits, int64_t n, const uint32_t* count_dev,
                                     const rr_key_params* p, void* stream);

/* ------------------------------------------------------------- coherence
 * Ray coherence measure M^64_CPS of Section 4.3 for n rays in the given
 * order.  Each group of 64 consecutive rays (the last may be shorter) gets
 * the surface area of a fitted capsule: its axis joins the centroid of the
 * origins and the centroid of the termination points, and the radii of its
 * two hemispheres and of the cone between them are the mean distances of the
 * origins, respectively the termination points, from that axis:
 *   2 pi r_o^2 + 2 pi r_t^2 + pi (r_o + r_t) sqrt(h^2 + (r_o - r_t)^2),
 * h the distance between the centroids (with coincident centroids the
 * distances are taken to that point).  hits[i] is the traced hit of rays[i];
 * a hit terminates at o + t d, a miss at o + min(tmax, E) d, E the largest
 * extent of p's box (p's other fields are not used).
 *  group_out device double[ceil(n / 64)]: the per-group areas.
 *  mean_out  device double: their mean (0 for n = 0).
 * Double precision; the sums differ from a sequential evaluation only by
 * rounding. */
rr_status rr_coherence_m64(const rr_ray* rays, const rr_hit* hits, int64_t n, const rr_key_params* p,
                           double* group_out, double* mean_out, void* stream);

/* ------------------------------------------------------------------- sort
 * Section 3.2: stable ascending radix sort of (key, index) pairs, in place.
 * The result is unique: the lexicographic order of (key, index) when the
 * input indices ascend (in general: by key, equal keys in input position
 * order).  rr_sort runs an LSD sort with 8-bit digits (one histogram pass,
 * then one stable scatter pass per digit).  n_max is the capacity; when count_dev
 * (device uint32) is given, only its first *count_dev pairs are sorted
 * (count_dev must not exceed n_max).  workspace (device, >= the size
 * reported by rr_sort_workspace_size, 256-byte aligned) is scratch that the
 * call overwrites.  The scatter passes are tuned for a device they have to
 * themselves: run beside other long kernels (other streams) they stay
 * correct but can be much slower; the batched layer (rr_batch.h) schedules
 * its sorts for sharing. */
rr_status rr_sort_workspace_size(int64_t n_max, uint32_t key_bits, size_t* bytes);
rr_status rr_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                  void* workspace, size_t ws_bytes, void* stream);
/* The most-significant-digit sort: two stable scatter passes on the two
 * highest 8-bit digits in which the keys differ, then every bucket of equal
 * top digits sorted on its other digits in LDS.  64-bit keys with n_max below
 * 2^27 (otherwise RR_ERR_UNSUPPORTED).  Arguments, workspace and result as
 * for rr_sort.  Faster than rr_sort when every bucket holds at most 512 keys
 * (evenly spread keys from about 2M to 17M pairs, where each bucket is sorted
 * by one wave); slower for clustered keys such as the paper's ray keys, whose
 * large buckets are sorted by whole blocks. */
rr_status rr_sort_msd(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                      void* workspace, size_t ws_bytes, void* stream);
/* The LSD sort with an explicit radix digit width (4 or 8 bits) and keys
 * per thread (tile size); every choice gives the identical result, that of
 * rr_sort.  rr_sort uses 8-bit digits and 8 keys per thread, 16 from 2^24
 * keys (n_max) on. */
rr_status rr_sort_ex(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                     uint32_t digit_bits, uint32_t keys_per_thread, void* workspace, size_t ws_bytes,
                     void* stream);

/* Local (block-wise) sorting of Section 3.2: every run of `block` consecutive
 * pairs (block = 1024, 2048 or 4096; the last run may be shorter) is sorted
 * on its own, in place, stably by unsigned key, so run r holds the pairs of
 * positions [r * block, (r + 1) * block) in (key, input position) order.
 * Cheaper than rr_sort, the resulting order is less coherent.  count_dev as
 * for rr_sort.  Needs no workspace.  RR_ERR_UNSUPPORTED for another block
 * size. */
rr_status rr_local_sort(void* keys, uint32_t* idx, int64_t n_max, const uint32_t* count_dev, uint32_t key_bits,
                        uint32_t block, void* stream);

/* ----------------------------------------------------------------- gather
 * Section 3.2, "an additional pass" that moves the ray data into key order:
 * out[i] = in[idx[i]] for i < n (n = *count_dev when given, else n_max).
 * in holds n_max rays and out n_max slots; they must not overlap.  An index
 * >= n_max yields an all-NaN record instead of a read outside `in`. */
rr_status rr_gather(const rr_ray* in, const uint32_t* idx, int64_t n_max, const uint32_t* count_dev, rr_ray* out,
                    void* stream);

/* Inverse of the gather for hits: out[idx[i]] = in[i] for i < n.  out holds
 * n_max slots; slots not named by idx are left untouched and indices
 * >= n_max are skipped. */
rr_status rr_scatter_hits(const rr_hit* in, const uint32_t* idx, int64_t n_max, const uint32_t* count_dev,
                          rr_hit* out, void* stream);

/* ------------------------------------------------------------------ trace
 * Closest hit of each ray (Section 4.1's nearest-hit kernel, here a
 * software stack traversal of the scene BVH with a two-sided
 * Moller-Trumbore triangle test in binary32).  The hit is the
 * lexicographic minimum of (t, prim) over the triangles whose test passes
 * with tmin < t < tmax, so it does not depend on ray order, BVH or launch
 * shape.  hits[i] belongs to rays[i] for i < n (n = *count_dev when
 * given).  Launches of up to about 98K rays (n_max; what one resident wave
 * of its blocks holds) on quantised nodes trace each ray with four lanes,
 * one child or triangle per lane; larger ones with one lane per ray in
 * persistent wavefronts.  Both give the same hits. */
rr_status rr_trace(rr_scene s, const rr_ray* rays, int64_t n_max, const uint32_t* count_dev, rr_hit* hits,
                   void* stream);
/* Any-hit (occlusion) trace, for shadow rays (Section 4 traces two shadow
 * rays per bounce): hits[i] is a miss {+inf, -1, 0, 0} when no triangle
 * meets ray i in (tmin, tmax), else the record {t, prim, u, v} of one such
 * triangle -- which one depends on the traversal, so callers should rely on
 * prim >= 0 only as "occluded" (the record is still exact for that
 * triangle).  Arguments as for rr_trace. */
rr_status rr_trace_any(rr_scene s, const rr_ray* rays, int64_t n_max, const uint32_t* count_dev, rr_hit* hits,
                       void* stream);

/* rr_trace in persistent wavefronts of one lane per ray at any size, with
 * an explicit lane-refill threshold (1..64): a wavefront loads new rays
 * into its idle lanes once at least `refill` lanes are idle (the traversal
 * shape the autotuner varies).  Same hits for every value. */
rr_status rr_trace_ex(rr_scene s, const rr_ray* rays, int64_t n_max, const uint32_t* count_dev, rr_hit* hits,
                      uint32_t refill, void* stream);

/* Profiling variant of rr_trace (Section 4.2 compares the control-flow
 * efficiency of the trace kernel on sorted and unsorted rays): same hits,
 * plus RR_TRACE_PROFILE_COUNTERS device uint64 counters written to stats_dev
 * (overwritten):
 *   [0] loop trips summed over rays, [1] loop trips of each wavefront x 64
 *       summed over wavefronts (so [0]/[1] is the SIMD efficiency),
 *   [2] inner-node visits, [3] leaf visits, [4] triangle tests, [5] rays,
 *   [6] the deepest traversal stack any ray reached (entries),
 *   [7] stack pushes beyond the 16 entries held in LDS (into scratch).
 * Slower than rr_trace (global atomics); for measurement only. */
#define RR_TRACE_PROFILE_COUNTERS 8
rr_status rr_trace_profile(rr_scene s, const rr_ray* rays, int64_t n, rr_hit* hits, uint64_t* stats_dev,
                           void* stream);

/* --------------------------------------------------------- fused pipeline
 * Keys (with compaction when `alive` is given), sort, gather and trace on
 * one stream: the reordered trace of Section 3.2 / Section 4.4.1.  With the
 * device-wide sort, the gather is done by the sort's last pass.
 *  hits      device, n entries.  With RR_HITS_ORIGINAL_ORDER, hits[i] is the
 *            hit of rays[i] and dead slots receive a miss record; otherwise
 *            hits[i] belongs to the i-th ray in key order and entries past
 *            the live count are untouched.
 *  perm_out  optional device uint32[n]: the sorted ray indices (identity for
 *            RR_KEY_NONE; compacted live indices when alive is given).
 *  count_out optional device uint32: the number of traced rays.
 *  workspace device scratch of at least rr_reorder_workspace_size bytes.
 * RR_KEY_NONE traces the (compacted) rays in their original order.
 * RR_KEY_TWO_POINT_ADAPTIVE computes its keys from the table p->aux and,
 * after the trace, adds the traced lengths to that table. */
#define RR_HITS_ORIGINAL_ORDER 1u
/* Trace through the sorted index instead of gathering the rays first
 * (Section 4.4.1, indirect ray access). */
#define RR_INDIRECT 2u
/* Sort locally (rr_local_sort) in runs of 1024, 2048 or 4096 keys instead of
 * device-wide; at most one of these. */
#define RR_LOCAL_SORT_1024 4u
#define RR_LOCAL_SORT_2048 8u
#define RR_LOCAL_SORT_4096 16u
/* Any-hit tracing (rr_trace_any) instead of closest-hit; refused
 * (RR_ERR_INVALID_ARGUMENT) with RR_KEY_TWO_POINT_ADAPTIVE, whose table
 * learns from closest hits. */
#define RR_ANY_HIT 32u
/* The device-wide sort is the most-significant-digit sort (rr_sort_msd)
 * instead of rr_sort's LSD sort: 64-bit keys and n below 2^27 (otherwise
 * RR_ERR_UNSUPPORTED); not with RR_LOCAL_SORT_* (RR_ERR_INVALID_ARGUMENT);
 * no effect with RR_KEY_NONE. */
#define RR_SORT_MSD 64u
rr_status rr_reorder_workspace_size(int64_t n_max, const rr_key_params* p, size_t* bytes);
rr_status rr_reorder_and_trace(rr_scene s, const rr_ray* rays, int64_t n, const uint8_t* alive,
                               const rr_key_params* p, rr_hit* hits, uint32_t* perm_out, uint32_t* count_out,
                               uint32_t flags, void* workspace, size_t ws_bytes, void* stream);

/* --------------------------------------------------- without allocation
 * For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation):
 * rr_reorder_and_trace with its workspace in a static device array of
 * RR_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  Arguments, results and errors are those of
 * rr_reorder_and_trace without the workspace; the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  A call whose
 * workspace (rr_reorder_workspace_size) exceeds the array is rejected with
 * RR_ERR_WORKSPACE_TOO_SMALL before anything is enqueued: the limit is
 * about 2.25M rays with 64-bit keys and 2.5M with 32-bit keys (or none).
 * All calls on one GPU share that GPU's array; every call initialises what
 * it reads, but calls that overlap on one GPU (other streams or threads
 * without ordering between them) race and must be serialised by the
 * caller.  The first call on a device looks the array's address up. */
#define RR_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)
rr_status rr_reorder_and_trace_noalloc(rr_scene s, const rr_ray* rays, int64_t n, const uint8_t* alive,
                                       const rr_key_params* p, rr_hit* hits, uint32_t* perm_out,
                                       uint32_t* count_out, uint32_t flags, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RR_H */
