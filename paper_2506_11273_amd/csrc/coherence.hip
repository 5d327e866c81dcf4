// Ray coherence measure M^64_CPS (Section 4.3): for each group of 64
// consecutive rays, the surface area of a capsule fitted to the group; its
// axis joins the centroid of the origins and the centroid of the
// termination points, and the radii of its two hemispheres (and of the cone
// between them) are the mean distances of the origins, respectively the
// termination points, from that axis:
//   2 pi r_o^2 + 2 pi r_t^2 + pi (r_o + r_t) sqrt(h^2 + (r_o - r_t)^2),
// h the distance between the centroids.  A hit terminates at o + t d, a miss
// at o + min(tmax, E) d (E the largest extent of the box).  One wave64 per
// group, double precision, sums by butterfly exchanges (every lane of a wave
// ends with the same sum); the mean over groups is a fixed-order reduction.
#include "common.hpp"

#pragma clang fp contract(off)

namespace rr {
namespace {

constexpr int kCpsBlock = 256;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

__global__ __launch_bounds__(kCpsBlock) void k_cps(const float4* __restrict__ rays, const float4* __restrict__ hits,
                                                   uint32_t n, float E, double* __restrict__ out) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t g = blockIdx.x * (kCpsBlock / kWave) + threadIdx.x / kWave;
  const uint32_t first = g * (uint32_t)kWave;
  if (first >= n) return;  // wave-uniform
  const uint32_t cnt = min((uint32_t)kWave, n - first);
  const bool ok = lane < cnt;
  double p[3] = {0.0, 0.0, 0.0}, t[3] = {0.0, 0.0, 0.0};
  if (ok) {
    const float4 a = rays[2 * (size_t)(first + lane)];
    const float4 b = rays[2 * (size_t)(first + lane) + 1];
    const float4 h = hits[first + lane];
    const double len = __float_as_int(h.y) >= 0 ? (double)h.x : (double)(b.w < E ? b.w : E);
    p[0] = a.x; p[1] = a.y; p[2] = a.z;
    t[0] = (double)a.x + len * (double)b.x;
    t[1] = (double)a.y + len * (double)b.y;
    t[2] = (double)a.z + len * (double)b.z;
  }
  const double c = (double)cnt;
  double co[3], ct[3], axis[3], h2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    co[k] = wave_sum(p[k]) / c;
    ct[k] = wave_sum(t[k]) / c;
    axis[k] = ct[k] - co[k];
    h2 += axis[k] * axis[k];
  }
  const double h = sqrt(h2);
  double dp[3], dt[3], sp = 0.0, st = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dp[k] = p[k] - co[k];
    dt[k] = t[k] - co[k];
  }
  if (h > 0.0) {
    double ap = 0.0, at = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ap += dp[k] * axis[k] / h;
      at += dt[k] * axis[k] / h;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double x = dp[k] - ap * axis[k] / h, y = dt[k] - at * axis[k] / h;
      sp += x * x;
      st += y * y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sp += dp[k] * dp[k];
      st += dt[k] * dt[k];
    }
  }
  const double ro = wave_sum(ok ? sqrt(sp) : 0.0) / c;
  const double rt = wave_sum(ok ? sqrt(st) : 0.0) / c;
  const double area = 2.0 * kPi * ro * ro + 2.0 * kPi * rt * rt + kPi * (ro + rt) * sqrt(h2 + (ro - rt) * (ro - rt));
  if (lane == 0) out[g] = area;
}

__global__ __launch_bounds__(1024) void k_mean(const double* __restrict__ v, uint32_t G, double* __restrict__ mean) {
  __shared__ double s[1024];
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < G; i += 1024) acc += v[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *mean = G ? s[0] / (double)G : 0.0;
}

}  // namespace

rr_status launch_coherence(const rr_ray* rays, const rr_hit* hits, int64_t n, float E, double* group_out,
                           double* mean_out, hipStream_t st) {
  const uint32_t G = (uint32_t)((n + kWave - 1) / kWave);
  if (G > 0) {
    const uint32_t blocks = (G + kCpsBlock / kWave - 1) / (kCpsBlock / kWave);
    hipLaunchKernelGGL(k_cps, dim3(blocks), dim3(kCpsBlock), 0, st, reinterpret_cast<const float4*>(rays),
                       reinterpret_cast<const float4*>(hits), (uint32_t)n, E, group_out);
  }
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(1024), 0, st, group_out, G, mean_out);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

}  // namespace rr
