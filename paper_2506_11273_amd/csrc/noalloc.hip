// rr_reorder_and_trace_noalloc: the fused reorder-and-trace call with its
// workspace in a static device array instead of caller memory, for callers
// that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid allocation).
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy from the time the code object is loaded until the
// process ends.  In host code its name only stands in for the symbol, so
// its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and only that address is handed to kernels.
// Every call on a GPU shares that GPU's array and leaves its contents
// behind; each kernel of the call initialises what it reads (histograms,
// look-back words and headers are cleared by the call's own setup kernels),
// so nothing depends on what a previous call left.  Calls that overlap on
// one GPU (other streams, other threads) race on the array.
#include <mutex>

#include "common.hpp"

namespace {

constexpr size_t kScratchBytes = RR_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up on the
// first call on the device), or nullptr with *st set on failure.
void* scratch_address(rr_status* st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    *st = RR_ERR_DEVICE;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      *st = RR_ERR_DEVICE;
      return nullptr;
    }
    g_ptr[dev] = ptr;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" rr_status rr_reorder_and_trace_noalloc(rr_scene s, const rr_ray* rays, int64_t n, const uint8_t* alive,
                                                  const rr_key_params* p, rr_hit* hits, uint32_t* perm_out,
                                                  uint32_t* count_out, uint32_t flags, void* stream) {
  if (!p) return RR_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  rr_status st = rr_reorder_workspace_size(n, p, &need);
  if (st != RR_OK) return st;
  if (need > kScratchBytes) return RR_ERR_WORKSPACE_TOO_SMALL;
  st = RR_OK;
  void* ptr = scratch_address(&st);
  if (!ptr) return st;
  return rr::reorder_and_trace_in_scratch(s, rays, n, alive, p, hits, perm_out, count_out, flags, ptr, kScratchBytes,
                                          stream);
}
