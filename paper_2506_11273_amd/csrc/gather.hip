// Ray-data reordering (Section 3.2: after the key/index sort "an additional
// pass" moves the ray records into key order; Section 4.4.1 measures it as
// the dominant overhead because its reads are incoherent) and the inverse
// scatter of hits.
//
// Two lanes move one 32-byte ray: each loads one 16-byte half, so a lane
// pair reads one contiguous 32-byte record and a wave writes 1 KiB of
// contiguous output.
#include "common.hpp"

namespace rr {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t read_count(const uint32_t* count_dev, uint32_t n_max) {
  if (!count_dev) return n_max;
  const uint32_t c = *count_dev;
  return c < n_max ? c : n_max;
}

__global__ __launch_bounds__(kBlock) void k_gather(const float4* __restrict__ in, const uint32_t* __restrict__ idx,
                                                   const uint32_t* count_dev, uint32_t n_max,
                                                   float4* __restrict__ out) {
  const uint32_t n = read_count(count_dev, n_max);
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t i = (uint32_t)(t >> 1), h = (uint32_t)(t & 1);
  if (i >= n) return;
  const uint32_t j = idx[i];
  // an index outside the input yields a NaN record instead of a stray read
  out[2 * (size_t)i + h] = j < n_max ? in[2 * (size_t)j + h] : make_float4(__int_as_float(0x7fc00000),
                                                                            __int_as_float(0x7fc00000),
                                                                            __int_as_float(0x7fc00000),
                                                                            __int_as_float(0x7fc00000));
}

__global__ __launch_bounds__(kBlock) void k_scatter_hits(const float4* __restrict__ in,
                                                         const uint32_t* __restrict__ idx, const uint32_t* count_dev,
                                                         uint32_t n_max, float4* __restrict__ out) {
  const uint32_t n = read_count(count_dev, n_max);
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = idx[i];
  if (j < n_max) out[j] = in[i];
}

__global__ __launch_bounds__(kBlock) void k_fill_miss(float4* __restrict__ out, uint32_t n) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  out[i] = make_float4(__int_as_float(0x7f800000), __int_as_float(-1), 0.0f, 0.0f);
}

__global__ __launch_bounds__(kBlock) void k_copy_u32(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                     const uint32_t* count_dev, uint32_t n_max) {
  const uint32_t n = read_count(count_dev, n_max);
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = in[i];
}

__global__ __launch_bounds__(kBlock) void k_iota(uint32_t* __restrict__ out, uint32_t n) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = i;
}

__global__ void k_set_u32(uint32_t* out, uint32_t n, uint32_t value) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) out[i] = value;
}

inline uint32_t blocks_for(uint64_t threads) { return (uint32_t)((threads + kBlock - 1) / kBlock); }

}  // namespace

rr_status launch_gather(const rr_ray* in, const uint32_t* idx, int64_t n_max, const uint32_t* count_dev, rr_ray* out,
                        hipStream_t st) {
  if (n_max <= 0) return RR_OK;
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(2 * (uint64_t)n_max)), dim3(kBlock), 0, st,
                     reinterpret_cast<const float4*>(in), idx, count_dev, (uint32_t)n_max,
                     reinterpret_cast<float4*>(out));
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status launch_scatter_hits(const rr_hit* in, const uint32_t* idx, int64_t n_max, const uint32_t* count_dev,
                              rr_hit* out, hipStream_t st) {
  if (n_max <= 0) return RR_OK;
  hipLaunchKernelGGL(k_scatter_hits, dim3(blocks_for((uint64_t)n_max)), dim3(kBlock), 0, st,
                     reinterpret_cast<const float4*>(in), idx, count_dev, (uint32_t)n_max,
                     reinterpret_cast<float4*>(out));
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status launch_fill_miss(rr_hit* out, int64_t n, hipStream_t st) {
  if (n <= 0) return RR_OK;
  hipLaunchKernelGGL(k_fill_miss, dim3(blocks_for((uint64_t)n)), dim3(kBlock), 0, st,
                     reinterpret_cast<float4*>(out), (uint32_t)n);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status launch_copy_u32(const uint32_t* in, uint32_t* out, int64_t n_max, const uint32_t* count_dev,
                          hipStream_t st) {
  if (n_max <= 0) return RR_OK;
  hipLaunchKernelGGL(k_copy_u32, dim3(blocks_for((uint64_t)n_max)), dim3(kBlock), 0, st, in, out, count_dev,
                     (uint32_t)n_max);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status launch_iota(uint32_t* out, int64_t n, hipStream_t st) {
  if (n <= 0) return RR_OK;
  hipLaunchKernelGGL(k_iota, dim3(blocks_for((uint64_t)n)), dim3(kBlock), 0, st, out, (uint32_t)n);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status launch_set_u32(uint32_t* out, uint32_t value, hipStream_t st) { return launch_fill_u32(out, 1, value, st); }

rr_status launch_fill_u32(uint32_t* out, uint32_t n, uint32_t value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(256), 0, st, out, n, value);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

}  // namespace rr
