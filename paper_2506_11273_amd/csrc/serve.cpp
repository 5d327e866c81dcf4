// Serving loop with continuous batching over the batched path.
//
// Requests (a device ray buffer, a key method and a device hit buffer) are
// submitted with an arrival time.  A scheduling thread admits arrived
// requests in arrival order into the batch forming for a free slot while
// they fit the slot's capacity, launches the batch on that slot's stream and
// records an event; a finished batch frees its slot, so requests that arrive
// while others run start as soon as a slot is free and their work overlaps
// on the device with the batches still running.  Slot workspaces are sized
// so that all of them together stay within the HBM budget.  A request
// asking for hits in ray order that is larger than the server's split size
// is served as consecutive parts of at most that many rays, each reordered
// and traced as a segment of its own: parts of one request can run on
// several slots at once and smaller requests fit in between, and since a
// ray's hit does not depend on which rays it is traced with, the hits equal
// those of the request traced alone.  Every request's hits come back in
// the order it asked for and equal those of the request traced alone.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "rr_batch.h"

namespace {

using clk = std::chrono::steady_clock;

struct Req {
  rr_request_stats st{};
  const rr_ray* rays = nullptr;
  rr_hit* hits = nullptr;
  rr_key_params key{};
  uint32_t flags = 0;  // hit order: RR_HITS_ORIGINAL_ORDER or key order
  int32_t parts_left = 0;
};

// A queued unit of work: rays [off, off + n) of a request.
struct Part {
  int64_t id;
  int64_t off, n;
  int64_t bytes;
};

struct Slot {
  rr_batch batch = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<int64_t> reqs;  // request of each part in the batch
  int64_t bytes = 0;
};

}  // namespace

struct rr_server_s {
  rr_scene scene = nullptr;
  int device = 0;
  rr_server_config cfg{};
  int64_t slot_bytes = 0;
  double bytes_per_ray = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;     // wakes the loop (new request, shutdown)
  std::condition_variable done_cv;  // wakes waiters
  std::condition_variable gone_cv;  // wakes rr_server_destroy when the last waiter has left
  int32_t waiters = 0;              // threads inside rr_server_wait / rr_server_drain
  std::deque<Part> pending;       // parts in arrival order
  std::unordered_map<int64_t, Req> reqs;
  int64_t next_id = 1;
  int64_t inflight_bytes = 0, peak_inflight = 0;
  int64_t batches = 0, rejected = 0;
  bool started = false, stop = false;
  clk::time_point t0;
  std::thread loop;
};

namespace {

bool device_ptr(const void* p, uintptr_t align) {
  if (!p || (reinterpret_cast<uintptr_t>(p) % align)) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

double now_s(rr_server sv) { return std::chrono::duration<double>(clk::now() - sv->t0).count(); }

// A batch finished: each of its parts is done; a request is done when its
// last part is (with the first error any part met).
void finish_slot(rr_server sv, Slot& s, rr_status status, double t) {
  for (int64_t id : s.reqs) {
    Req& r = sv->reqs[id];
    if (status != RR_OK && r.st.status == RR_OK) r.st.status = status;
    if (--r.parts_left == 0) {
      r.st.done = 1;
      r.st.finish_s = t;
    }
  }
  sv->inflight_bytes -= s.bytes;
  s.reqs.clear();
  s.bytes = 0;
  s.busy = false;
}

// Queues the parts of request id behind every part that arrived no later.
void insert_by_arrival(rr_server sv, int64_t id, const std::vector<Part>& parts) {
  const double a = sv->reqs[id].st.arrival_s;
  auto it = sv->pending.end();
  while (it != sv->pending.begin() && sv->reqs[(it - 1)->id].st.arrival_s > a) --it;
  sv->pending.insert(it, parts.begin(), parts.end());
}

void run_loop(rr_server sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  std::vector<rr_segment> segs;
  while (true) {
    const double t = now_s(sv);
    bool any_busy = false;
    // completions
    for (Slot& s : sv->slots) {
      if (!s.busy) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipSuccess) {
        finish_slot(sv, s, RR_OK, t);
        sv->done_cv.notify_all();
      } else if (q != hipErrorNotReady) {
        (void)hipGetLastError();
        finish_slot(sv, s, RR_ERR_DEVICE, t);
        sv->done_cv.notify_all();
      } else {
        any_busy = true;
      }
    }
    if (sv->stop && !any_busy) break;
    // admission and launch on free slots
    for (Slot& s : sv->slots) {
      if (s.busy || sv->stop) continue;
      int64_t rays = 0;
      uint32_t flags = 0;
      segs.clear();
      while (!sv->pending.empty() && (int32_t)segs.size() < sv->cfg.max_batch_requests) {
        const Part pt = sv->pending.front();
        Req& r = sv->reqs[pt.id];
        if (r.st.arrival_s > t) break;  // not yet arrived
        if (rays + pt.n > sv->cfg.max_batch_rays) break;
        // one hit order per batch: a request asking for the other order
        // starts the next batch
        if (!segs.empty() && r.flags != flags) break;
        flags = r.flags;
        segs.push_back(rr_segment{r.rays + pt.off, r.hits + pt.off, nullptr, pt.n, r.key});
        s.reqs.push_back(pt.id);
        s.bytes += pt.bytes;
        rays += pt.n;
        sv->pending.pop_front();
      }
      if (segs.empty()) continue;
      rr_status st = rr_batch_run(s.batch, segs.data(), (int32_t)segs.size(), flags, s.stream);
      if (st == RR_OK && hipEventRecord(s.done, s.stream) != hipSuccess) st = RR_ERR_DEVICE;
      const double ts = now_s(sv);
      for (int64_t id : s.reqs) {
        Req& r = sv->reqs[id];
        if (r.st.start_s < 0) r.st.start_s = ts;  // the first part's launch
        r.st.batch_requests = (int32_t)segs.size();
      }
      sv->inflight_bytes += s.bytes;
      sv->peak_inflight = std::max(sv->peak_inflight, sv->inflight_bytes);
      ++sv->batches;
      if (st != RR_OK) {
        finish_slot(sv, s, st, ts);
        sv->done_cv.notify_all();
      } else {
        s.busy = true;
        any_busy = true;
      }
    }
    // wait: poll quickly while the device works, else sleep until the next
    // arrival or a new submission
    if (any_busy) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else if (!sv->pending.empty()) {
      const double next = sv->reqs[sv->pending.front().id].st.arrival_s;
      const double wait = std::max(0.0, next - now_s(sv));
      sv->cv.wait_for(lk, std::chrono::duration<double>(std::min(wait, 0.05)));
    } else {
      sv->cv.wait_for(lk, std::chrono::milliseconds(50));
    }
  }
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = p * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

rr_status rr_server_create(rr_scene s, const rr_server_config* cfg, rr_server* out) {
  if (!out) return RR_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!s || !cfg || cfg->slots < 1 || cfg->slots > 16 || cfg->max_batch_rays <= 0 ||
      cfg->max_batch_rays >= RR_MAX_RAYS || cfg->max_batch_requests < 1 || cfg->max_batch_requests > 4096 ||
      cfg->hbm_budget_bytes <= 0 || cfg->split_rays < 0 || cfg->split_rays > cfg->max_batch_rays)
    return RR_ERR_INVALID_ARGUMENT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->d.device) return RR_ERR_INVALID_ARGUMENT;
  rr_server sv = new (std::nothrow) rr_server_s;
  if (!sv) return RR_ERR_OUT_OF_MEMORY;
  sv->scene = s;
  sv->device = dev;
  sv->cfg = *cfg;
  rr_status st = RR_OK;
  for (int32_t k = 0; k < cfg->slots && st == RR_OK; ++k) {
    Slot sl;
    st = rr_batch_create(s, cfg->max_batch_rays, cfg->max_batch_requests, nullptr, &sl.batch);
    if (st != RR_OK) break;
    int64_t bytes = 0;
    (void)rr_batch_info(sl.batch, &bytes, nullptr);
    if ((int64_t)(k + 1) * bytes > cfg->hbm_budget_bytes) {
      (void)rr_batch_destroy(sl.batch);
      if (k == 0) st = RR_ERR_BUDGET;  // not even one slot fits
      break;
    }
    sv->slot_bytes = bytes;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      (void)rr_batch_destroy(sl.batch);
      st = RR_ERR_DEVICE;
      break;
    }
    sv->slots.push_back(sl);
  }
  if (st != RR_OK) {
    for (Slot& sl : sv->slots) {
      (void)rr_batch_destroy(sl.batch);
      (void)hipStreamDestroy(sl.stream);
      (void)hipEventDestroy(sl.done);
    }
    delete sv;
    return st;
  }
  sv->bytes_per_ray = (double)sv->slot_bytes / (double)cfg->max_batch_rays;
  sv->t0 = clk::now();
  *out = sv;
  return RR_OK;
}

rr_status rr_server_start(rr_server sv) {
  if (!sv) return RR_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->started) return RR_ERR_INVALID_ARGUMENT;
  sv->t0 = clk::now();
  sv->started = true;
  try {
    sv->loop = std::thread(run_loop, sv);
  } catch (...) {
    sv->started = false;
    return RR_ERR_DEVICE;
  }
  return RR_OK;
}

rr_status rr_server_submit(rr_server sv, const rr_ray* rays, int64_t n, const rr_key_params* key, rr_hit* hits,
                           uint32_t flags, double arrival_s, int64_t* id) {
  if (!sv || !key || !id || n < 0 || (flags & ~RR_HITS_ORIGINAL_ORDER)) return RR_ERR_INVALID_ARGUMENT;
  if (key->kind != RR_KEY_NONE) {
    rr::KeyPlan p;
    const rr_status st = rr::make_key_plan(key, &p);
    if (st != RR_OK) return st;
    if (p.aux && !device_ptr(p.aux, 16)) return RR_ERR_INVALID_ARGUMENT;
  }
  // a bad request is refused here so that it never fails its batch-mates
  if (n > 0 && (!device_ptr(rays, 16) || !device_ptr(hits, 16))) return RR_ERR_INVALID_ARGUMENT;
  // parts: only a request in ray order is split (its hits do not depend on
  // the split); an empty request is one empty part.  Every part must fit a
  // batch.
  const int64_t split = sv->cfg.split_rays;
  const int64_t part = (flags & RR_HITS_ORIGINAL_ORDER) && split > 0 && n > split ? split : std::max<int64_t>(n, 1);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (part > sv->cfg.max_batch_rays) {
    ++sv->rejected;
    return RR_ERR_BUDGET;
  }
  Req r;
  r.st.id = sv->next_id++;
  r.st.n = n;
  r.st.arrival_s = arrival_s >= 0 ? arrival_s : now_s(sv);
  r.st.start_s = -1.0;
  r.rays = rays;
  r.hits = hits;
  r.key = *key;
  r.flags = flags;
  std::vector<Part> parts;
  for (int64_t off = 0; off == 0 || off < n; off += part) {
    const int64_t m = std::min(part, n - off);
    parts.push_back(Part{r.st.id, off, m, (int64_t)(sv->bytes_per_ray * (double)m)});
  }
  r.parts_left = (int32_t)parts.size();
  sv->reqs[r.st.id] = r;
  insert_by_arrival(sv, r.st.id, parts);
  *id = r.st.id;
  sv->cv.notify_all();
  return RR_OK;
}

// Counts a thread inside rr_server_wait / rr_server_drain (under the
// mutex), so that rr_server_destroy frees the server only after every such
// thread has left it.
struct WaiterGuard {
  rr_server sv;
  explicit WaiterGuard(rr_server s) : sv(s) { ++sv->waiters; }
  ~WaiterGuard() {
    if (--sv->waiters == 0) sv->gone_cv.notify_all();
  }
};

rr_status rr_server_wait(rr_server sv, int64_t id, double timeout_s, rr_request_stats* out) {
  if (!sv) return RR_ERR_INVALID_ARGUMENT;
  std::unique_lock<std::mutex> lk(sv->mu);
  WaiterGuard guard(sv);  // destroyed before lk, with the mutex held
  auto it = sv->reqs.find(id);
  if (it == sv->reqs.end()) return RR_ERR_INVALID_ARGUMENT;
  const auto deadline = clk::now() + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(timeout_s));
  while (!sv->reqs[id].st.done)
    if (sv->done_cv.wait_until(lk, deadline) == std::cv_status::timeout && !sv->reqs[id].st.done)
      return RR_ERR_DEVICE;
  if (out) *out = sv->reqs[id].st;
  return sv->reqs[id].st.status;
}

rr_status rr_server_drain(rr_server sv, double timeout_s) {
  if (!sv) return RR_ERR_INVALID_ARGUMENT;
  std::unique_lock<std::mutex> lk(sv->mu);
  WaiterGuard guard(sv);
  const auto deadline = clk::now() + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(timeout_s));
  auto all_done = [&] {
    for (auto& kv : sv->reqs)
      if (!kv.second.st.done) return false;
    return true;
  };
  while (!all_done())
    if (sv->done_cv.wait_until(lk, deadline) == std::cv_status::timeout && !all_done()) return RR_ERR_DEVICE;
  return RR_OK;
}

rr_status rr_server_stats_get(rr_server sv, rr_server_stats* out) {
  if (!sv || !out) return RR_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(sv->mu);
  rr_server_stats s{};
  std::vector<double> lat;
  double first = 1e300, last = 0;
  for (auto& kv : sv->reqs) {
    const rr_request_stats& r = kv.second.st;
    if (!r.done) continue;
    if (r.status != RR_OK) {
      ++s.failed;
      continue;
    }
    ++s.completed;
    s.rays += r.n;
    lat.push_back((r.finish_s - r.arrival_s) * 1e3);
    first = std::min(first, r.arrival_s);
    last = std::max(last, r.finish_s);
  }
  s.rejected = sv->rejected;
  s.p50_ms = percentile(lat, 0.50);
  s.p99_ms = percentile(lat, 0.99);
  double sum = 0, mx = 0;
  for (double v : lat) {
    sum += v;
    mx = std::max(mx, v);
  }
  s.mean_ms = lat.empty() ? 0 : sum / (double)lat.size();
  s.max_ms = mx;
  s.wall_s = lat.empty() ? 0 : last - first;
  s.mrays_per_s = s.wall_s > 0 ? (double)s.rays / s.wall_s / 1e6 : 0;
  s.batches = sv->batches;
  s.peak_inflight_bytes = sv->peak_inflight;
  *out = s;
  return RR_OK;
}

rr_status rr_server_destroy(rr_server sv) {
  if (!sv) return RR_ERR_INVALID_ARGUMENT;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  if (sv->loop.joinable()) sv->loop.join();
  {
    // requests never launched end as failed, so no waiter is left behind
    std::lock_guard<std::mutex> lk(sv->mu);
    for (const Part& pt : sv->pending) {
      sv->reqs[pt.id].st.done = 1;
      sv->reqs[pt.id].st.status = RR_ERR_DEVICE;
    }
    sv->pending.clear();
  }
  {
    // every request is done now: threads still in rr_server_wait or
    // rr_server_drain return; the server is freed only after they have left
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->done_cv.notify_all();
    sv->gone_cv.wait(lk, [&] { return sv->waiters == 0; });
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(sv->device);
  for (Slot& sl : sv->slots) {
    (void)hipStreamSynchronize(sl.stream);
    (void)rr_batch_destroy(sl.batch);
    (void)hipStreamDestroy(sl.stream);
    (void)hipEventDestroy(sl.done);
  }
  (void)hipSetDevice(cur);
  delete sv;
  return RR_OK;
}

}  // extern "C"
