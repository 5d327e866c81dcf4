// Closest-hit trace: software stack traversal of the scene's binary BVH with
// a two-sided Moller-Trumbore triangle test in binary32 (the nearest-hit
// kernel of Section 4.1; the paper's method is agnostic to the trace kernel,
// Section 1).
//
// Result definition: the lexicographic minimum of (t, primitive id) over the
// triangles whose test passes with tmin < t < tmax.  The triangle test is
// evaluated in a fixed operation order without contraction, so a given
// (ray, triangle) pair always yields the same bits; the box test is
// conservative (zero direction components are nudged to a tiny value and the
// far distance gets a small relative slack), so pruning never removes the
// defining minimum and the result does not depend on ray order or launch
// shape.
//
// Layout: an inner node is 4 x float4 = 64 bytes holding both children's
// boxes, (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y), (c1.lo.x, c1.hi.x, c1.lo.y,
// c1.hi.y), (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z), (child0, child1, -, -).
// A child >= 0 is an inner node; a child < 0 is a leaf ~(first << 3 | count).
// A triangle is 3 x float4 = 48 bytes: (v0, e1.x), (e1.yz, e2.xy),
// (e2.z, prim id bits, -, -), with e1 = v1 - v0 and e2 = v2 - v0.
// The per-lane stack lives in LDS, interleaved by lane.
#include "common.hpp"

#pragma clang fp contract(off)

namespace rr {
namespace {

constexpr int kTraceBlock = 256;
constexpr float kFarSlack = 0x1p-16f;
constexpr float kTinyDir = 1e-20f;

__device__ __forceinline__ uint32_t read_count(const uint32_t* count_dev, uint32_t n_max) {
  if (!count_dev) return n_max;
  const uint32_t c = *count_dev;
  return c < n_max ? c : n_max;
}

__device__ __forceinline__ float nudge(float d) { return fabsf(d) < kTinyDir ? copysignf(kTinyDir, d) : d; }

// Slab test of one child box; returns the entry distance in *tn.
__device__ __forceinline__ bool slab(float lox, float hix, float loy, float hiy, float loz, float hiz, float ox,
                                     float oy, float oz, float ix, float iy, float iz, float tmin, float tbest,
                                     float* tn) {
  const float ax = (lox - ox) * ix, bx = (hix - ox) * ix;
  const float ay = (loy - oy) * iy, by = (hiy - oy) * iy;
  const float az = (loz - oz) * iz, bz = (hiz - oz) * iz;
  const float n = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), tmin));
  float f = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tbest));
  f = __builtin_fmaf(fabsf(f), kFarSlack, f);
  *tn = n;
  return n <= f;
}

// Counters of the profiling variant (Section 4.2 profiles control-flow
// efficiency): lane loop trips, wave loop trips x 64, inner-node visits,
// leaf visits, triangle tests, rays.
struct TraceStats {
  unsigned long long lane_trips, wave_trips64, inner, leaves, tri_tests, rays;
};

__device__ void trace_stats_flush(TraceStats* st, uint32_t trips, uint32_t inner, uint32_t leaves, uint32_t tris,
                                  uint32_t ray) {
  // wave maximum of the trips (the wave runs until its longest lane ends)
  uint32_t mx = trips;
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, kWave));
  atomicAdd(&st->lane_trips, (unsigned long long)trips);
  atomicAdd(&st->inner, (unsigned long long)inner);
  atomicAdd(&st->leaves, (unsigned long long)leaves);
  atomicAdd(&st->tri_tests, (unsigned long long)tris);
  atomicAdd(&st->rays, (unsigned long long)ray);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&st->wave_trips64, 64ull * mx);
}

template <bool STATS>
__global__ __launch_bounds__(kTraceBlock) void k_trace(const float4* __restrict__ nodes,
                                                       const float4* __restrict__ tris, int32_t root,
                                                       const float4* __restrict__ rays,
                                                       const uint32_t* __restrict__ idx, const uint32_t* count_dev,
                                                       uint32_t n_max, float4* __restrict__ hits,
                                                       TraceStats* stats) {
  __shared__ int32_t s_stack[kTraceStack * kTraceBlock];
  const uint32_t n = read_count(count_dev, n_max);
  const uint32_t i = blockIdx.x * kTraceBlock + threadIdx.x;
  if (!STATS && i >= n) return;
  // the profiling variant keeps every lane to the end for its wave reductions
  const uint32_t r = i < n ? (idx ? idx[i] : i) : 0u;
  const bool live = i < n && r < n_max;
  if (i < n && !live) hits[i] = make_float4(__int_as_float(0x7f800000), __int_as_float(-1), 0.0f, 0.0f);
  uint32_t trips = 0, n_inner = 0, n_leaf = 0, n_tri = 0;
  if (live) {
    const float4 ra = rays[2 * (size_t)r];
    const float4 rb = rays[2 * (size_t)r + 1];
    const float ox = ra.x, oy = ra.y, oz = ra.z, tmin = ra.w;
    const float dx = rb.x, dy = rb.y, dz = rb.z;
    const float ix = 1.0f / nudge(dx), iy = 1.0f / nudge(dy), iz = 1.0f / nudge(dz);

    float tbest = rb.w;
    int32_t bprim = -1;
    float bu = 0.0f, bv = 0.0f;

    int32_t* stack = s_stack + threadIdx.x;
    int sp = 0;
    int32_t node = root;
    while (true) {
      if (STATS) ++trips;
      if (node >= 0) {
        if (STATS) ++n_inner;
        const float4* N = nodes + 4 * (size_t)node;
        const float4 n0 = N[0], n1 = N[1], n2 = N[2];
        const int4 n3 = *reinterpret_cast<const int4*>(N + 3);
        float t0, t1;
        const bool h0 = slab(n0.x, n0.y, n0.z, n0.w, n2.x, n2.y, ox, oy, oz, ix, iy, iz, tmin, tbest, &t0);
        const bool h1 = slab(n1.x, n1.y, n1.z, n1.w, n2.z, n2.w, ox, oy, oz, ix, iy, iz, tmin, tbest, &t1);
        if (h0 && h1) {
          const bool first0 = t0 <= t1;
          // sp never exceeds the tree depth, which the builder caps at kTraceStack
          if (sp < kTraceStack) {
            stack[sp * kTraceBlock] = first0 ? n3.y : n3.x;
            ++sp;
          }
          node = first0 ? n3.x : n3.y;
          continue;
        }
        if (h0 || h1) {
          node = h0 ? n3.x : n3.y;
          continue;
        }
      } else {
        const int32_t code = ~node;
        const int32_t first = code >> 3, count = code & 7;
        if (STATS) {
          ++n_leaf;
          n_tri += count;
        }
        for (int32_t k = 0; k < count; ++k) {
          const float4* T = tris + 3 * (size_t)(first + k);
          const float4 a = T[0], b = T[1], c = T[2];
          const float e1x = a.w, e1y = b.x, e1z = b.y;
          const float e2x = b.z, e2y = b.w, e2z = c.x;
          const int32_t prim = __float_as_int(c.y);
          const float sx = ox - a.x, sy = oy - a.y, sz = oz - a.z;
          const float px = dy * e2z - dz * e2y;
          const float py = dz * e2x - dx * e2z;
          const float pz = dx * e2y - dy * e2x;
          const float det = (e1x * px + e1y * py) + e1z * pz;
          if (det == 0.0f) continue;
          const float inv = 1.0f / det;
          const float u = ((sx * px + sy * py) + sz * pz) * inv;
          if (!(u >= 0.0f && u <= 1.0f)) continue;
          const float qx = sy * e1z - sz * e1y;
          const float qy = sz * e1x - sx * e1z;
          const float qz = sx * e1y - sy * e1x;
          const float v = ((dx * qx + dy * qy) + dz * qz) * inv;
          if (!(v >= 0.0f && u + v <= 1.0f)) continue;
          const float t = ((e2x * qx + e2y * qy) + e2z * qz) * inv;
          if (t > tmin && (t < tbest || (t == tbest && prim < bprim))) {
            tbest = t;
            bprim = prim;
            bu = u;
            bv = v;
          }
        }
      }
      if (sp == 0) break;
      --sp;
      node = stack[sp * kTraceBlock];
    }
    hits[i] = make_float4(bprim >= 0 ? tbest : __int_as_float(0x7f800000), __int_as_float(bprim), bu, bv);
  }
  if (STATS) trace_stats_flush(stats, trips, n_inner, n_leaf, n_tri, live ? 1u : 0u);
}

}  // namespace

rr_status launch_trace(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                       const uint32_t* count_dev, rr_hit* hits, hipStream_t st) {
  if (n_max <= 0) return RR_OK;
  const uint32_t blocks = (uint32_t)((n_max + kTraceBlock - 1) / kTraceBlock);
  hipLaunchKernelGGL(k_trace<false>, dim3(blocks), dim3(kTraceBlock), 0, st, s.nodes, s.tris, s.root,
                     reinterpret_cast<const float4*>(rays), idx, count_dev, (uint32_t)n_max,
                     reinterpret_cast<float4*>(hits), nullptr);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

rr_status launch_trace_stats(const DeviceScene& s, const rr_ray* rays, int64_t n_max, rr_hit* hits,
                             uint64_t* stats_dev, hipStream_t st) {
  if (n_max <= 0) return RR_OK;
  const uint32_t blocks = (uint32_t)((n_max + kTraceBlock - 1) / kTraceBlock);
  hipLaunchKernelGGL(k_trace<true>, dim3(blocks), dim3(kTraceBlock), 0, st, s.nodes, s.tris, s.root,
                     reinterpret_cast<const float4*>(rays), nullptr, nullptr, (uint32_t)n_max,
                     reinterpret_cast<float4*>(hits), reinterpret_cast<TraceStats*>(stats_dev));
  RR_LAUNCH_CHECK();
  return RR_OK;
}

}  // namespace rr
