/*
 * rr_batch.h -- batched and served ray reordering + tracing on MI355X.
 *
 * The per-call path of rr.h (keys of Section 3.1, the key/index sort and
 * ray gather of Section 3.2, the closest-hit trace of Section 4.1) applied
 * to many wavefronts at once, and a serving loop on top of it.  Conventions
 * are those of rr.h: extern "C", rr_status results, device pointers owned
 * by the caller, work enqueued on the given stream.
 */
#ifndef RR_BATCH_H
#define RR_BATCH_H

#include "rr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ batch
 * One segment = one wavefront: n rays at `rays` (device), reordered with
 * its own key method and traced.  Hits go to `hits` (device, n entries): in
 * ray order with RR_HITS_ORIGINAL_ORDER, else in the segment's key order.
 * perm (device, nullable, n entries) receives the segment-local sorted ray
 * indices.  Per segment the results equal those of rr_reorder_and_trace on
 * that wavefront alone, bit for bit.  Every key kind may be used; a
 * RR_KEY_TWO_POINT_ADAPTIVE segment reads its length table (key.aux) but the
 * batch does not add its traced lengths to it (rr_length_table_accumulate
 * does), so segments sharing a table see the same estimates. */
typedef struct rr_segment {
  const rr_ray* rays;
  rr_hit* hits;
  uint32_t* perm;
  int64_t n;
  rr_key_params key;
} rr_segment;

/* Launch shape of a batch: radix digit width (4 or 8 bits), keys per
 * thread of a sort tile (8 or 16), the trace's lane-refill threshold
 * (1..64), the trace kernel's block size (128, 256 or 512 threads; the
 * closest-hit trace on quantised nodes, the other scenes trace with 256),
 * and the order in which the sort's scatter passes take tiles:
 * RR_TILES_COUNTER (0, the default) hands them out from a counter, so a
 * tile is only awaited while a running block holds it, which keeps the
 * decoupled look-back from its slow fallback when other kernels share the
 * device (the server's concurrent batches); RR_TILES_FIXED (1) gives block
 * b the tiles b, b + G, ... with no counter atomics, faster for a batch
 * that has the device to itself.  Results do not depend on the shape. */
#define RR_TILES_COUNTER 0u
#define RR_TILES_FIXED 1u
typedef struct rr_batch_config {
  uint32_t digit_bits;
  uint32_t keys_per_thread;
  uint32_t refill;
  uint32_t tile_order;
  uint32_t trace_block;
} rr_batch_config;

typedef struct rr_batch_s* rr_batch;

/* Run the batch as individual kernel launches instead of the captured
 * graph (for comparison and debugging). */
#define RR_BATCH_EAGER 0x100u

/* Creates a batch for up to max_rays rays in up to max_segments segments
 * against scene s (same device).  Allocates its device buffers (about
 * 100 bytes per ray of capacity, see rr_batch_info) and a capture stream;
 * cfg may be NULL for the default shape.  A batch runs one batch at a time:
 * concurrent runs need separate batch objects. */
rr_status rr_batch_create(rr_scene s, int64_t max_rays, int32_t max_segments, const rr_batch_config* cfg,
                          rr_batch* out);
rr_status rr_batch_info(rr_batch b, int64_t* device_bytes, rr_batch_config* cfg);
rr_status rr_batch_set_config(rr_batch b, const rr_batch_config* cfg);

/* Reorders and traces every segment: one descriptor upload and one graph
 * launch on `stream` (the graph for the current shape is captured on first
 * use).  flags: RR_HITS_ORIGINAL_ORDER, RR_BATCH_EAGER.  The total ray count
 * must not exceed max_rays (RR_ERR_BUDGET otherwise). */
rr_status rr_batch_run(rr_batch b, const rr_segment* segs, int32_t nseg, uint32_t flags, void* stream);

/* Times every launch shape on this batch of segments (reps runs each,
 * median) and keeps the fastest; returns it and its time.  Synchronises.
 * It runs the batch alone, so it may choose RR_TILES_FIXED: a batch that
 * will share the device should keep RR_TILES_COUNTER. */
rr_status rr_batch_autotune(rr_batch b, const rr_segment* segs, int32_t nseg, int32_t reps, rr_batch_config* best,
                            float* best_ms, void* stream);
rr_status rr_batch_destroy(rr_batch b);

/* ---------------------------------------------------------------- serving
 * A request loop with continuous batching: submitted requests wait until
 * their arrival time, are admitted while their workspace fits the HBM
 * budget, and are packed into batches that run on `slots` streams, so new
 * requests start while earlier ones are still on the device.  Latency is
 * measured from arrival to the moment the loop sees the batch finish. */
typedef struct rr_server_config {
  int32_t slots;             /* concurrent batches (streams), >= 1 */
  int64_t hbm_budget_bytes;  /* device memory the server may hold for batch workspaces */
  int64_t max_batch_rays;    /* largest batch (and largest request or part) */
  int32_t max_batch_requests;  /* segments (requests or parts) per batch */
  int64_t split_rays;        /* 0, or (at most max_batch_rays): a request in ray order larger
                                than this is served as consecutive parts of at most split_rays
                                rays, each reordered and traced as a segment of its own (its
                                hits do not change) */
} rr_server_config;

typedef struct rr_request_stats {
  int64_t id;
  int64_t n;
  int32_t status;        /* RR_OK, or the error that failed the request */
  int32_t done;
  double arrival_s;      /* seconds since rr_server_start */
  double start_s;        /* launched on the device */
  double finish_s;       /* completion seen by the loop */
  int32_t batch_requests;
} rr_request_stats;

typedef struct rr_server_stats {
  int64_t completed, failed, rejected, rays;
  double p50_ms, p99_ms, mean_ms, max_ms;
  double wall_s;         /* first arrival to last completion */
  double mrays_per_s;
  int64_t batches;
  int64_t peak_inflight_bytes;
} rr_server_stats;

typedef struct rr_server_s* rr_server;

rr_status rr_server_create(rr_scene s, const rr_server_config* cfg, rr_server* out);
/* Starts the clock that arrival times refer to and the scheduling thread. */
rr_status rr_server_start(rr_server sv);
/* Queues a request (no device work in the call).  arrival_s < 0 means now.
 * flags: RR_HITS_ORIGINAL_ORDER (hits[i] belongs to rays[i]) or 0 (hits in
 * the request's key order); a batch holds requests of one hit order.
 * A request larger than max_batch_rays is rejected with RR_ERR_BUDGET,
 * unless it is served as parts (each of at most split_rays rays).
 * The rays must be complete in device memory when rr_server_submit is
 * called: the server's streams read them without waiting for the stream
 * that produced them.  The ray and hit buffers must stay valid until the
 * request is done. */
rr_status rr_server_submit(rr_server sv, const rr_ray* rays, int64_t n, const rr_key_params* key, rr_hit* hits,
                           uint32_t flags, double arrival_s, int64_t* id);
/* Blocks until the request is done (or timeout_s passes: RR_ERR_DEVICE).
 * rr_server_destroy fails every request not yet launched, waits for the
 * launched ones, and returns only after every thread blocked in
 * rr_server_wait or rr_server_drain has returned. */
rr_status rr_server_wait(rr_server sv, int64_t id, double timeout_s, rr_request_stats* out);
/* Blocks until every submitted request is done. */
rr_status rr_server_drain(rr_server sv, double timeout_s);
rr_status rr_server_stats_get(rr_server sv, rr_server_stats* out);
rr_status rr_server_destroy(rr_server sv);

#ifdef __cplusplus
}
#endif
#endif /* RR_BATCH_H */
