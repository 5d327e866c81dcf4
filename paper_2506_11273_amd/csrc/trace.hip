// Closest-hit trace: software stack traversal of a 4-wide BVH with a
// two-sided Moller-Trumbore triangle test in binary32 (the nearest-hit
// kernel of Section 4.1; the paper's method is agnostic to the trace kernel,
// Section 1).  The any-hit variant (the shadow rays of Section 4) stops a
// ray at the first triangle it finds in (tmin, tmax).
//
// Result definition: the lexicographic minimum of (t, primitive id) over the
// triangles whose test passes with tmin < t < tmax.  The triangle test is
// evaluated in a fixed operation order without contraction, so a given
// (ray, triangle) pair always yields the same bits; the box test is
// conservative (zero direction components are nudged to a tiny value and the
// far distance gets a small relative slack), so pruning never removes the
// defining minimum and the result does not depend on ray order, BVH or
// launch shape.
//
// Layout: a 4-wide inner node is either 8 x float4 = 128 bytes holding its
// four child boxes in SoA form (lo.x[4], hi.x[4], lo.y[4], hi.y[4], lo.z[4],
// hi.z[4], child[4], unused), or 4 x float4 = 64 bytes with the child bounds
// quantised to 8 bits against the node box: (p.xyz, s.z),
// (lo.x, hi.x, lo.y, hi.y as 4 bytes each), (lo.z, hi.z, s.x, s.y), child[4],
// with power-of-two steps s; a bound decodes to the exact p + q * s, codes
// chosen by the builder so that these planes enclose the child box.  A child
// >= 0 is an inner node, kEmptyChild an unused slot, and a child < 0 a leaf
// ~(first << 3 | count) of at most 7 triangles (the builder makes at most 3).
// A triangle is 3 x float4 = 48 bytes: (v0, e1.x), (e1.yz, e2.xy),
// (e2.z, prim id bits, -, -), with e1 = v1 - v0 and e2 = v2 - v0.
//
// Execution: persistent wavefronts.  Each XCD owns a contiguous share of
// the ray slots (in key order when the rays were reordered); its blocks take
// packets of that share in turn (16 to 64 slots, chosen per launch), and a
// wave refills its idle lanes from its block's packets whenever at least
// `refill` lanes are idle, so lanes whose rays finish early do not idle until
// the wave's longest ray ends, the waves of a block run out of rays together,
// and the rays in flight on an XCD stay a window of neighbouring slots.
// A wave alternates between an inner-node loop and a leaf loop (while-while
// traversal, a found leaf postponed while the lane goes on with inner nodes).
// Neither loop runs until its last lane is done: the inner loop ends once at
// most kLoopExit lanes still need an inner node to find a leaf, the leaf
// loop once at most kLoopExit lanes still hold a leaf; those lanes carry
// their state into the wave's next round, so the few long traversals of a
// wave do not keep the other 60 lanes idle.
// The traversal stack holds at most 3 entries per tree level; its first
// kLdsStack entries live in LDS (interleaved by lane), the rest in scratch.
#include <algorithm>

#include "common.hpp"

#pragma clang fp contract(off)

namespace rr {
namespace {

constexpr float kFarSlack = 0x1p-16f;
constexpr float kTinyDir = 1e-20f;
constexpr int kLdsStack = 16;
constexpr int kSpillStack = kTraceStack4 - kLdsStack;
// Packets are 2^pshift consecutive ray slots (16 to 64, chosen per launch;
// see launch4q).
constexpr int kLoopExit = 8;      // lanes left in a loop when the wave moves on

__device__ __forceinline__ uint32_t read_count(const uint32_t* count_dev, uint32_t n_max) {
  if (!count_dev) return n_max;
  const uint32_t c = *count_dev;
  return c < n_max ? c : n_max;
}

__device__ __forceinline__ float nudge(float d) { return fabsf(d) < kTinyDir ? copysignf(kTinyDir, d) : d; }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Counters of the profiling variant (Section 4.2 profiles control-flow
// efficiency): active lane iterations, wave iterations x 64, inner-node
// visits, leaf visits, triangle tests, rays; then the deepest traversal
// stack any ray reached and the number of pushes that went to the scratch
// part of the stack (entries beyond the LDS part).
struct TraceStats {
  unsigned long long lane_trips, wave_trips64, inner, leaves, tri_tests, rays, max_depth, spill_pushes;
};

struct Ray {
  float ox, oy, oz, tmin;
  float dx, dy, dz, tmax;
  float ix, iy, iz;
  float ax, ay, az;  // |inv| * 2^-20 per axis (exact scalings)
};

// Slab test of one child box; *tn receives the entry distance.
__device__ __forceinline__ bool slab(float lx, float hx, float ly, float hy, float lz, float hz, const Ray& R,
                                     float tbest, float* tn) {
  const float ax = (lx - R.ox) * R.ix, bx = (hx - R.ox) * R.ix;
  const float ay = (ly - R.oy) * R.iy, by = (hy - R.oy) * R.iy;
  const float az = (lz - R.oz) * R.iz, bz = (hz - R.oz) * R.iz;
  const float n = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), R.tmin));
  float f = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tbest));
  f = __builtin_fmaf(fabsf(f), kFarSlack, f);
  *tn = n;
  return n <= f;
}

// Ray distances to the near and far planes of the four children of a
// quantised node along one axis, in ray-relative form: with delta = p - o,
// a plane q lies at t = q * (s * inv) + delta * inv, one fused multiply-add
// per plane.  Which of the node's two code words holds the near planes
// depends only on the sign of inv, so the caller passes the words in
// near/far order.  Every plane is moved outward by
// ei = (|delta| 2^-20 + s 2^-12) |inv| (the near planes toward the ray, the
// far planes away from it: near base delta*inv - ei, far base
// delta*inv + ei), computed as fma(|delta|, |inv| 2^-20, |s*inv| 2^-12)
// with exact power-of-two scalings, so it falls short of that value by at
// most a factor 1 - 2^-22.  The rounding of delta, of delta*inv, of the
// bases, of s*inv and of the final fused multiply-add is below
// (|delta| + 128 s) |inv| 2^-22, about a quarter of the move, so the
// computed slab contains the slab of the decoded box, which contains the
// child's box.  (Coordinates are below 1e18 and steps below 2^61, so
// nothing overflows.)
__device__ __forceinline__ void qaxis(float p, float s, float o, float inv, float ainv20, uint32_t wnear,
                                      uint32_t wfar, float (&tn)[4], float (&tf)[4]) {
  const float delta = p - o;
  const float step = s * inv;
  const float ei = __builtin_fmaf(fabsf(delta), ainv20, fabsf(step) * 0x1p-12f);
  const float di = delta * inv;
  const float nb = di - ei;
  const float fb = di + ei;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    tn[j] = __builtin_fmaf((float)((wnear >> (8 * j)) & 0xFFu), step, nb);
    tf[j] = __builtin_fmaf((float)((wfar >> (8 * j)) & 0xFFu), step, fb);
  }
}

// Slab test from near and far plane distances (see qaxis).
__device__ __forceinline__ bool qslab(float nx, float fx, float ny, float fy, float nz, float fz, float tmin,
                                      float tbest, float* tn) {
  const float n = fmaxf(fmaxf(nx, ny), fmaxf(nz, tmin));
  float f = fminf(fminf(fx, fy), fminf(fz, tbest));
  f = __builtin_fmaf(fabsf(f), kFarSlack, f);
  *tn = n;
  return n <= f;
}

__device__ __forceinline__ void cswap(float& ta, int32_t& ca, float& tb, int32_t& cb) {
  const bool s = tb < ta;
  const float t = s ? tb : ta;
  tb = s ? ta : tb;
  ta = t;
  const int32_t c = s ? cb : ca;
  cb = s ? ca : cb;
  ca = c;
}

template <int BLOCK, bool STATS, bool QNODE, bool ANY>
__global__ __launch_bounds__(BLOCK) void k_trace4(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                                  int32_t root, const float4* __restrict__ rays,
                                                  const uint32_t* __restrict__ idx, const uint32_t* count_dev,
                                                  uint32_t n_max, float4* __restrict__ hits, uint32_t refill,
                                                  uint32_t pshift, TraceStats* stats) {
  __shared__ int32_t s_stack[kLdsStack * BLOCK];
  int32_t spill[kSpillStack];
  const uint32_t n = read_count(count_dev, n_max);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t waves = gridDim.x * (BLOCK / kWave);
  // Workgroups are dispatched to the XCDs round-robin; renumber them so that
  // each XCD works on one contiguous share of the rays, which keeps the part
  // of the BVH its L2 must hold small when the rays are spatially sorted.
  const uint32_t nb = gridDim.x, q = nb / kXcds, rem = nb % kXcds;
  const uint32_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
  const uint32_t xb0 = x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;  // XCD's first block
  const uint32_t xbn = x < rem ? q + 1 : q;                                    // and its block count
  const uint32_t wpb = BLOCK / kWave;
  // The XCD's share of the ray slots is [xs, xe), cut into packets of
  // 2^pshift slots.  With W waves on the XCD, wpb per block, the block whose
  // first wave is w0 holds packets k W + w0 .. k W + w0 + wpb - 1 for k = 0,
  // 1, ... (as if wave w took packets w, w + W, w + 2W, ...), so the blocks of
  // an XCD move through the share together and the rays in flight on it at
  // any time are a window of consecutive slots.  The block's waves take its
  // rays in that order from a counter in LDS, as many at a time as they have
  // idle lanes: a wave whose rays finish early takes more, and the block's
  // waves run out of rays together instead of each after a fixed share.
  const uint32_t W = xbn * wpb, w0 = j * wpb;
  const uint32_t xs = (uint32_t)(((uint64_t)xb0 * wpb * n) / waves);
  const uint32_t xe = (uint32_t)(((uint64_t)(xb0 + xbn) * wpb * n) / waves);
  // slot of the block's v-th ray (monotonic in v)
  const uint32_t pk = 1u << pshift;
  auto slot_of = [&](uint32_t v) -> uint64_t {
    const uint32_t q = v >> pshift;
    return (uint64_t)xs + ((uint64_t)(q / wpb) * W + w0 + q % wpb) * pk + (v & (pk - 1));
  };
  __shared__ uint32_t s_taken;  // rays the block's waves have taken
  if (threadIdx.x == 0) s_taken = 0;
  __syncthreads();
  int32_t* lstack = s_stack + threadIdx.x;

  Ray R{};
  int32_t slot = -1;  // ray slot this lane works on, -1 when idle
  int32_t node = 0;   // next node to visit: inner node, leaf code, or kEmptyChild when none is left
  int32_t leaf = 0;   // postponed leaf code, 0 when none
  int sp = 0;
  float tbest = 0.0f, bu = 0.0f, bv = 0.0f;
  int32_t bprim = -1;
  unsigned long long st_trips = 0, st_wave = 0, st_inner = 0, st_leaf = 0, st_tri = 0, st_rays = 0;
  unsigned long long st_depth = 0, st_spill = 0;

  while (true) {
    // ---- refill idle lanes from the block's packets (wave-uniform decision)
    const uint64_t idle = __ballot(slot < 0);
    const uint32_t n_idle = (uint32_t)__popcll(idle);
    const bool more = slot_of(__hip_atomic_load(&s_taken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) < xe;
    if (n_idle == kWave && !more) break;
    if (more && (n_idle >= refill || n_idle == kWave)) {
      // one lane takes n_idle rays for the wave (another wave may have
      // taken the last ones since the check: lanes past the share stay idle)
      const int first = __builtin_ctzll(__ballot(1));
      uint32_t base = 0;
      if ((int)lane == first) base = atomicAdd(&s_taken, n_idle);
      base = __shfl(base, first, kWave);
      if (slot < 0) {
        const uint64_t s64 = slot_of(base + lanes_below(idle));
        if (s64 < xe) {
          const uint32_t s = (uint32_t)s64;
          slot = (int32_t)s;
          const uint32_t r = idx ? idx[s] : s;
          if (r < n_max) {
            const float4 a = rays[2 * (size_t)r];
            const float4 b = rays[2 * (size_t)r + 1];
            R.ox = a.x; R.oy = a.y; R.oz = a.z; R.tmin = a.w;
            R.dx = b.x; R.dy = b.y; R.dz = b.z; R.tmax = b.w;
            R.ix = 1.0f / nudge(b.x);
            R.iy = 1.0f / nudge(b.y);
            R.iz = 1.0f / nudge(b.z);
            R.ax = fabsf(R.ix) * 0x1p-20f;
            R.ay = fabsf(R.iy) * 0x1p-20f;
            R.az = fabsf(R.iz) * 0x1p-20f;
            tbest = b.w;
            node = root;
          } else {
            // an index outside the rays: report a miss without tracing
            tbest = __int_as_float(0x7f800000);
            node = kEmptyChild;
          }
          bprim = -1;
          bu = bv = 0.0f;
          sp = 0;
          leaf = 0;
          if (STATS) ++st_rays;
        }
      }
    }
    // counts one wave iteration per wave (by the lowest active lane)
    auto wave_tick = [&]() {
      if (STATS) {
        if ((int)lane == __builtin_ctzll(__ballot(1))) ++st_wave;
      }
    };
    // While no lane of the wave has spilled (the common case, decided
    // wave-uniformly) a pop is a plain LDS read, not a load through a
    // generic pointer.
    auto pop_or_none = [&]() -> int32_t {
      if (sp == 0) return kEmptyChild;
      --sp;
      if (!__ballot(sp >= kLdsStack)) return lstack[sp * BLOCK];
      return sp < kLdsStack ? lstack[sp * BLOCK] : spill[sp - kLdsStack];
    };
    if (slot < 0) continue;

    // ---- inner nodes, until all but kLoopExit lanes hold a postponed leaf
    // (or has finished), so that node tests and triangle tests do not
    // diverge within one iteration
    while (node >= 0 && node != kEmptyChild) {
      wave_tick();
      if (STATS) {
        ++st_trips;
        ++st_inner;
      }
      float t0, t1, t2, t3;
      bool h0, h1, h2, h3;
      int4 cc;
      float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
      if constexpr (QNODE) {
        const float4* N = nodes + 4 * (size_t)node;
        const float4 a = N[0], b = N[1], c = N[2];
        cc = *reinterpret_cast<const int4*>(N + 3);
        const uint32_t xl = __float_as_uint(b.x), xh = __float_as_uint(b.y);
        const uint32_t yl = __float_as_uint(b.z), yh = __float_as_uint(b.w);
        const uint32_t zl = __float_as_uint(c.x), zh = __float_as_uint(c.y);
        qaxis(a.x, c.z, R.ox, R.ix, R.ax, R.ix < 0.0f ? xh : xl, R.ix < 0.0f ? xl : xh, lox, hix);
        qaxis(a.y, c.w, R.oy, R.iy, R.ay, R.iy < 0.0f ? yh : yl, R.iy < 0.0f ? yl : yh, loy, hiy);
        qaxis(a.z, a.w, R.oz, R.iz, R.az, R.iz < 0.0f ? zh : zl, R.iz < 0.0f ? zl : zh, loz, hiz);
        h0 = qslab(lox[0], hix[0], loy[0], hiy[0], loz[0], hiz[0], R.tmin, tbest, &t0) && cc.x != kEmptyChild;
        h1 = qslab(lox[1], hix[1], loy[1], hiy[1], loz[1], hiz[1], R.tmin, tbest, &t1) && cc.y != kEmptyChild;
        h2 = qslab(lox[2], hix[2], loy[2], hiy[2], loz[2], hiz[2], R.tmin, tbest, &t2) && cc.z != kEmptyChild;
        h3 = qslab(lox[3], hix[3], loy[3], hiy[3], loz[3], hiz[3], R.tmin, tbest, &t3) && cc.w != kEmptyChild;
      } else {
        const float4* N = nodes + 8 * (size_t)node;
        const float4 lx = N[0], hx = N[1], ly = N[2], hy = N[3], lz = N[4], hz = N[5];
        cc = *reinterpret_cast<const int4*>(N + 6);
        h0 = slab(lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, R, tbest, &t0) && cc.x != kEmptyChild;
        h1 = slab(lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, R, tbest, &t1) && cc.y != kEmptyChild;
        h2 = slab(lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, R, tbest, &t2) && cc.z != kEmptyChild;
        h3 = slab(lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, R, tbest, &t3) && cc.w != kEmptyChild;
      }
      const int m = (int)h0 + (int)h1 + (int)h2 + (int)h3;
      const float inf = __int_as_float(0x7f800000);
      float d0 = h0 ? t0 : inf, d1 = h1 ? t1 : inf, d2 = h2 ? t2 : inf, d3 = h3 ? t3 : inf;
      int32_t c0 = cc.x, c1 = cc.y, c2 = cc.z, c3 = cc.w;
      // nearest first; misses (inf) sort last
      cswap(d0, c0, d1, c1);
      cswap(d2, c2, d3, c3);
      cswap(d0, c0, d2, c2);
      cswap(d1, c1, d3, c3);
      cswap(d1, c1, d2, c2);
      if (!__ballot(sp + 3 > kLdsStack)) {
        // no lane can reach the scratch part (decided wave-uniformly):
        // every lane reads the entry below its top and writes three slots
        // from its top, without a branch.  With hits the m - 1 farther
        // ones go to sp.. (farthest deepest; the slots above the new top
        // receive copies that are never read) and the nearest is next;
        // without, the entry below the top is popped.
        const int32_t below = lstack[(sp > 0 ? sp - 1 : 0) * BLOCK];
        lstack[sp * BLOCK] = m == 4 ? c3 : (m == 3 ? c2 : c1);
        lstack[(sp + 1) * BLOCK] = m == 4 ? c2 : c1;
        lstack[(sp + 2) * BLOCK] = c1;
        node = m > 0 ? c0 : (sp > 0 ? below : kEmptyChild);
        sp = m > 0 ? sp + m - 1 : (sp > 0 ? sp - 1 : 0);
      } else if (m > 0) {
        const int32_t cs[3] = {c1, c2, c3};
#pragma unroll
        for (int k = 2; k >= 0; --k) {
          if (k + 1 < m) {
            if (sp < kLdsStack) lstack[sp * BLOCK] = cs[k];
            else spill[sp - kLdsStack] = cs[k];
            if (STATS && sp >= kLdsStack) ++st_spill;
            ++sp;
          }
        }
        node = c0;
      } else {
        node = pop_or_none();
      }
      if (STATS && (unsigned long long)sp > st_depth) st_depth = (unsigned long long)sp;
      if (node < 0 && leaf == 0) {
        leaf = node;
        node = pop_or_none();
      }
      if (__popcll(__ballot(leaf == 0 && node >= 0 && node != kEmptyChild)) <= kLoopExit) break;
    }
    if (node < 0 && leaf == 0) {
      leaf = node;
      node = pop_or_none();
    }

    // ---- the postponed leaf, then any leaves that follow on the stack
    while (leaf < 0) {
      wave_tick();
      const int32_t code = ~leaf;
      const int32_t first = code >> 3, count = code & 7;
      if (STATS) {
        ++st_trips;
        ++st_leaf;
        st_tri += (unsigned long long)count;
      }
      for (int32_t k = 0; k < count; ++k) {
        const float4* T = tris + 3 * (size_t)(first + k);
        const float4 a = T[0], b = T[1], c = T[2];
        const float e1x = a.w, e1y = b.x, e1z = b.y;
        const float e2x = b.z, e2y = b.w, e2z = c.x;
        const int32_t prim = __float_as_int(c.y);
        const float sx = R.ox - a.x, sy = R.oy - a.y, sz = R.oz - a.z;
        const float px = R.dy * e2z - R.dz * e2y;
        const float py = R.dz * e2x - R.dx * e2z;
        const float pz = R.dx * e2y - R.dy * e2x;
        const float det = (e1x * px + e1y * py) + e1z * pz;
        // every quantity is computed and the tests are combined into one
        // predicate: the lanes of a wave test different triangles, so early
        // exits would seldom skip work and only add branches (det = 0 gives
        // an infinite or NaN u, which the predicate rejects as well)
        const float inv = 1.0f / det;
        const float u = ((sx * px + sy * py) + sz * pz) * inv;
        const float qx = sy * e1z - sz * e1y;
        const float qy = sz * e1x - sx * e1z;
        const float qz = sx * e1y - sy * e1x;
        const float v = ((R.dx * qx + R.dy * qy) + R.dz * qz) * inv;
        const float t = ((e2x * qx + e2y * qy) + e2z * qz) * inv;
        const bool inside = det != 0.0f && u >= 0.0f && u <= 1.0f && v >= 0.0f && u + v <= 1.0f;
        if (inside && t > R.tmin && (t < tbest || (t == tbest && prim < bprim))) {
          tbest = t;
          bprim = prim;
          bu = u;
          bv = v;
          if constexpr (ANY) break;  // any occluder ends the ray
        }
      }
      leaf = 0;
      if constexpr (ANY) {
        if (bprim >= 0) {
          node = kEmptyChild;
          sp = 0;
        }
      }
      if (node < 0) {
        leaf = node;
        node = pop_or_none();
      }
      if (__popcll(__ballot(leaf < 0)) <= kLoopExit) break;
    }
    // a lane is done when its stack is empty and no leaf is left to test
    if (node == kEmptyChild && leaf == 0) {
      hits[slot] = make_float4(bprim >= 0 ? tbest : __int_as_float(0x7f800000), __int_as_float(bprim), bu, bv);
      slot = -1;
    }
  }
  if (STATS) {
    atomicAdd(&stats->lane_trips, st_trips);
    atomicAdd(&stats->inner, st_inner);
    atomicAdd(&stats->leaves, st_leaf);
    atomicAdd(&stats->tri_tests, st_tri);
    atomicAdd(&stats->rays, st_rays);
    atomicAdd(&stats->wave_trips64, 64ull * st_wave);
    atomicMax(&stats->max_depth, st_depth);
    atomicAdd(&stats->spill_pushes, st_spill);
  }
}

// ---------------------------------------------------------------------------
// The same trace with four lanes per ray, for launches too small to fill the
// device: with one ray per lane such a launch leaves most SIMDs with one wave
// or none, and its time is the latency of its longest traversals.  Here the
// four lanes of a quad share a ray and its state; lane q tests child q of
// each inner node (and triangles q, q + 4, ... of each leaf), so a node visit
// takes about half the issue time.  The quad orders the children it hit by
// entry distance (ties by child slot) with cross-lane moves inside the quad,
// pushes the farther ones and goes on with the nearest; the traversal stack
// lives in LDS whole.  Control flow is uniform within a quad, so every
// cross-lane move reads active lanes.  Box and triangle tests are those of
// k_trace4 (the same operations in the same order), so the hits are the
// same; the any-hit variant reports the (t, id)-least occluder of the first
// leaf that has one.
constexpr int kQuadBlock = 256;
constexpr int kQuadRays = kQuadBlock / 4;  // rays per block
constexpr int kQuadExit = 2;               // quads left in a loop when the wave moves on

// Cross-lane moves inside a quad (lane i reads lane i ^ m).
__device__ __forceinline__ int32_t quad_xor1(int32_t x) { return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ int32_t quad_xor2(int32_t x) { return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false); }
__device__ __forceinline__ int32_t quad_xor3(int32_t x) { return __builtin_amdgcn_update_dpp(0, x, 0x1B, 0xF, 0xF, false); }
__device__ __forceinline__ float quad_xor1(float x) { return __int_as_float(quad_xor1(__float_as_int(x))); }
__device__ __forceinline__ float quad_xor2(float x) { return __int_as_float(quad_xor2(__float_as_int(x))); }
__device__ __forceinline__ float quad_xor3(float x) { return __int_as_float(quad_xor3(__float_as_int(x))); }

// Distances to the near and far planes of one child (byte `sh / 8` of the
// code words) along one axis: qaxis for a single child.
__device__ __forceinline__ void qaxis1(float p, float s, float o, float inv, float ainv20, uint32_t wnear,
                                       uint32_t wfar, uint32_t sh, float* tn, float* tf) {
  const float delta = p - o;
  const float step = s * inv;
  const float ei = __builtin_fmaf(fabsf(delta), ainv20, fabsf(step) * 0x1p-12f);
  const float di = delta * inv;
  *tn = __builtin_fmaf((float)((wnear >> sh) & 0xFFu), step, di - ei);
  *tf = __builtin_fmaf((float)((wfar >> sh) & 0xFFu), step, di + ei);
}

// (t, id) of lane pairs: the lexicographically smaller, with its u, v.
__device__ __forceinline__ void quad_min(float& t, int32_t& id, float& u, float& v, float ot, int32_t oid, float ou,
                                         float ov) {
  const bool take = ot < t || (ot == t && oid < id);
  t = take ? ot : t;
  id = take ? oid : id;
  u = take ? ou : u;
  v = take ? ov : v;
}

template <int BLOCK, bool ANY>
__global__ __launch_bounds__(BLOCK) void k_trace_quad(const float4* __restrict__ nodes,
                                                      const float4* __restrict__ tris, int32_t root,
                                                      const float4* __restrict__ rays,
                                                      const uint32_t* __restrict__ idx, const uint32_t* count_dev,
                                                      uint32_t n_max, float4* __restrict__ hits) {
  constexpr int kRays = BLOCK / 4;
  __shared__ int32_t s_stack[kTraceStack4 * kRays];
  const uint32_t n = read_count(count_dev, n_max);
  const uint32_t q = threadIdx.x & 3u;
  const uint32_t rb = threadIdx.x >> 2;
  const uint32_t slot = blockIdx.x * (uint32_t)kRays + rb;
  if (slot >= n) return;  // whole quads leave together
  const uint32_t quad_shift = (threadIdx.x & (kWave - 1)) & ~3u;
  int32_t* stack = s_stack + rb;  // entry e at stack[e * kRays]

  Ray R{};
  float tbest = __int_as_float(0x7f800000), bu = 0.0f, bv = 0.0f;
  int32_t bprim = -1;
  int32_t node = kEmptyChild, leaf = 0;
  int sp = 0;
  const uint32_t r = idx ? idx[slot] : slot;
  if (r < n_max) {
    const float4 a = rays[2 * (size_t)r];
    const float4 b = rays[2 * (size_t)r + 1];
    R.ox = a.x; R.oy = a.y; R.oz = a.z; R.tmin = a.w;
    R.dx = b.x; R.dy = b.y; R.dz = b.z; R.tmax = b.w;
    R.ix = 1.0f / nudge(b.x);
    R.iy = 1.0f / nudge(b.y);
    R.iz = 1.0f / nudge(b.z);
    R.ax = fabsf(R.ix) * 0x1p-20f;
    R.ay = fabsf(R.iy) * 0x1p-20f;
    R.az = fabsf(R.iz) * 0x1p-20f;
    tbest = b.w;
    node = root;
  }
  auto pop_or_none = [&]() -> int32_t {
    if (sp == 0) return kEmptyChild;
    --sp;
    return stack[sp * kRays];
  };
  const uint32_t sh = 8u * q;
  const float inf = __int_as_float(0x7f800000);

  while (true) {
    // ---- inner nodes, until all but kQuadExit quads hold a postponed leaf
    while (node >= 0 && node != kEmptyChild) {
      const float4* N = nodes + 4 * (size_t)node;
      const float4 a = N[0], b = N[1], c = N[2];
      const int4 cc = *reinterpret_cast<const int4*>(N + 3);
      const int32_t child = q == 0 ? cc.x : q == 1 ? cc.y : q == 2 ? cc.z : cc.w;
      const uint32_t xl = __float_as_uint(b.x), xh = __float_as_uint(b.y);
      const uint32_t yl = __float_as_uint(b.z), yh = __float_as_uint(b.w);
      const uint32_t zl = __float_as_uint(c.x), zh = __float_as_uint(c.y);
      float nx, fx, ny, fy, nz, fz, tn;
      qaxis1(a.x, c.z, R.ox, R.ix, R.ax, R.ix < 0.0f ? xh : xl, R.ix < 0.0f ? xl : xh, sh, &nx, &fx);
      qaxis1(a.y, c.w, R.oy, R.iy, R.ay, R.iy < 0.0f ? yh : yl, R.iy < 0.0f ? yl : yh, sh, &ny, &fy);
      qaxis1(a.z, a.w, R.oz, R.iz, R.az, R.iz < 0.0f ? zh : zl, R.iz < 0.0f ? zl : zh, sh, &nz, &fz);
      const bool hit = qslab(nx, fx, ny, fy, nz, fz, R.tmin, tbest, &tn) && child != kEmptyChild;
      // rank among the quad's hits: nearer first, ties by child slot
      const float key = hit ? tn : inf;
      const float k1 = quad_xor1(key), k2 = quad_xor2(key), k3 = quad_xor3(key);
      const uint32_t q1 = q ^ 1u, q2 = q ^ 2u, q3 = q ^ 3u;
      const int rank = (int)(k1 < key || (k1 == key && q1 < q)) + (int)(k2 < key || (k2 == key && q2 < q)) +
                       (int)(k3 < key || (k3 == key && q3 < q));
      const int m = (int)__popcll((__ballot(hit) >> quad_shift) & 0xFull);
      if (m > 0) {
        // the farther hits onto the stack, farthest deepest; the nearest is next
        if (hit && rank >= 1) stack[(sp + m - 1 - rank) * kRays] = child;
        sp += m - 1;
        int32_t c0 = (hit && rank == 0) ? child : 0;
        c0 |= quad_xor1(c0);
        c0 |= quad_xor2(c0);
        node = c0;
      } else {
        node = pop_or_none();
      }
      if (node < 0 && leaf == 0) {
        leaf = node;
        node = pop_or_none();
      }
      if (__popcll(__ballot(leaf == 0 && node >= 0 && node != kEmptyChild)) <= 4 * kQuadExit) break;
    }
    if (node < 0 && leaf == 0) {
      leaf = node;
      node = pop_or_none();
    }

    // ---- leaves: lane q tests triangles q, q + 4, ...; the quad keeps the least (t, id)
    while (leaf < 0) {
      const int32_t code = ~leaf;
      const int32_t first = code >> 3, count = code & 7;
      float lt = tbest, lu = bu, lv = bv;
      int32_t lp = bprim;
      for (int32_t k = (int32_t)q; k < count; k += 4) {
        const float4* T = tris + 3 * (size_t)(first + k);
        const float4 a = T[0], b = T[1], c = T[2];
        const float e1x = a.w, e1y = b.x, e1z = b.y;
        const float e2x = b.z, e2y = b.w, e2z = c.x;
        const int32_t prim = __float_as_int(c.y);
        const float sx = R.ox - a.x, sy = R.oy - a.y, sz = R.oz - a.z;
        const float px = R.dy * e2z - R.dz * e2y;
        const float py = R.dz * e2x - R.dx * e2z;
        const float pz = R.dx * e2y - R.dy * e2x;
        const float det = (e1x * px + e1y * py) + e1z * pz;
        if (det == 0.0f) continue;
        const float inv = 1.0f / det;
        const float u = ((sx * px + sy * py) + sz * pz) * inv;
        if (!(u >= 0.0f && u <= 1.0f)) continue;
        const float qx = sy * e1z - sz * e1y;
        const float qy = sz * e1x - sx * e1z;
        const float qz = sx * e1y - sy * e1x;
        const float v = ((R.dx * qx + R.dy * qy) + R.dz * qz) * inv;
        if (!(v >= 0.0f && u + v <= 1.0f)) continue;
        const float t = ((e2x * qx + e2y * qy) + e2z * qz) * inv;
        if (t > R.tmin && (t < lt || (t == lt && prim < lp))) {
          lt = t;
          lp = prim;
          lu = u;
          lv = v;
        }
      }
      quad_min(lt, lp, lu, lv, quad_xor1(lt), quad_xor1(lp), quad_xor1(lu), quad_xor1(lv));
      quad_min(lt, lp, lu, lv, quad_xor2(lt), quad_xor2(lp), quad_xor2(lu), quad_xor2(lv));
      tbest = lt;
      bprim = lp;
      bu = lu;
      bv = lv;
      leaf = 0;
      if constexpr (ANY) {
        if (bprim >= 0) {  // any occluder ends the ray
          node = kEmptyChild;
          sp = 0;
        }
      }
      if (node < 0) {
        leaf = node;
        node = pop_or_none();
      }
      if (__popcll(__ballot(leaf < 0)) <= 4 * kQuadExit) break;
    }
    // a quad is done when its stack is empty and no leaf is left to test
    if (node == kEmptyChild && leaf == 0) {
      if (q == 0)
        hits[slot] = make_float4(bprim >= 0 ? tbest : __int_as_float(0x7f800000), __int_as_float(bprim), bu, bv);
      return;
    }
  }
}

// Rays of one resident wave of k_trace_quad blocks (LDS bounds it to about
// six blocks per CU).  Launches up to this size go to k_trace_quad
// (quantised nodes, closest and any hit): beyond it the blocks run in
// rounds and the one-lane kernel is as fast or faster.  Larger launches and
// every batch take k_trace4.
int64_t quad_capacity() {
  static const int64_t cached = [] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_trace_quad<kQuadBlock, false>, kQuadBlock, 0) !=
            hipSuccess ||
        per <= 0)
      per = 1;
    return (int64_t)cus * per * kQuadRays;
  }();
  return cached;
}

template <bool ANY>
rr_status launch_quad(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                      const uint32_t* count_dev, rr_hit* hits, hipStream_t st) {
  const uint32_t blocks = (uint32_t)((n_max + kQuadRays - 1) / kQuadRays);
  hipLaunchKernelGGL((k_trace_quad<kQuadBlock, ANY>), dim3(blocks), dim3(kQuadBlock), 0, st, s.nodes, s.tris, s.root,
                     reinterpret_cast<const float4*>(rays), idx, count_dev, (uint32_t)n_max,
                     reinterpret_cast<float4*>(hits));
  RR_LAUNCH_CHECK();
  return RR_OK;
}

constexpr int kTraceBlock = 256;

// Blocks of one resident wave of the grid, queried once per instance (a
// function-local static, so a server thread and the caller's thread may
// both ask).
template <int BLOCK, bool STATS, bool QNODE, bool ANY>
uint32_t resident_blocks() {
  static const uint32_t cached = [] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_trace4<BLOCK, STATS, QNODE, ANY>, BLOCK, 0) !=
            hipSuccess ||
        per <= 0)
      per = 1024 / BLOCK;
    return (uint32_t)(cus * per);
  }();
  return cached;
}

template <int BLOCK, bool STATS, bool QNODE, bool ANY>
rr_status launch4q(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                   const uint32_t* count_dev, rr_hit* hits, uint32_t refill, TraceStats* stats, hipStream_t st) {
  // enough waves to fill the device, but at least one full wave of rays each
  const uint64_t waves_needed = (uint64_t)(n_max + kWave - 1) / kWave;
  const uint64_t blocks_needed = (waves_needed + BLOCK / kWave - 1) / (BLOCK / kWave);
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(blocks_needed, resident_blocks<BLOCK, STATS, QNODE, ANY>());
  // Packet size.  A block's work is the sum over its packets, and the
  // launch ends with its slowest block.  In key order neighbouring rays cost
  // alike, so a block needs enough packets for their costs to even out,
  // while larger packets keep a wave's rays together.  The choice is about
  // 16 packets per wave: the power of two nearest in ratio, within 16 to 64
  // slots.  Measured on city wavefronts: at ~250 rays per wave (1080p),
  // 16-slot packets trace Two Point order 7-11% faster than 64-slot ones,
  // with pixel and shuffled order within 1-2%; at ~1,000 rays per wave
  // (2160p), 64 slots beat 16, 8 and 4 by 1-11%.  About 8 packets per wave
  // was within 2% (faster in key and shuffled order, slower in pixel order).
  const uint64_t waves = (uint64_t)blocks * (BLOCK / kWave);
  const uint64_t per_wave = ((uint64_t)n_max + waves - 1) / waves;
  uint32_t pshift = 4;
  while (pshift < 6 && per_wave * 5 >= (uint64_t)113 << pshift) ++pshift;  // per_wave / 2^pshift >= 16 sqrt 2
  // Refill threshold when the caller leaves it to the launch (0): 16, and 24
  // from 512 rays per wave on.  Measured against 16 on city wavefronts: at
  // ~1,000 rays per wave (2160p) 24 traced Two Point order ~3% faster and
  // pixel order ~1%, shuffled rays 0.5% slower; at ~250 rays per wave (1080p)
  // it was within 1%.
  if (refill == 0) refill = per_wave >= 512 ? 24u : kDefaultRefill;
  hipLaunchKernelGGL((k_trace4<BLOCK, STATS, QNODE, ANY>), dim3(blocks), dim3(BLOCK), 0, st, s.nodes, s.tris, s.root,
                     reinterpret_cast<const float4*>(rays), idx, count_dev, (uint32_t)n_max,
                     reinterpret_cast<float4*>(hits), refill, pshift, stats);
  RR_LAUNCH_CHECK();
  return RR_OK;
}

template <bool STATS, bool ANY = false>
rr_status launch4(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                  const uint32_t* count_dev, rr_hit* hits, uint32_t refill, TraceStats* stats, hipStream_t st,
                  uint32_t block = kTraceBlock) {
  if (n_max <= 0) return RR_OK;
  if (refill > (uint32_t)kWave) refill = kWave;  // 0: chosen per launch (launch4q)
  // the other block sizes exist for the closest-hit trace on quantised nodes
  if (!STATS && !ANY && s.quantised && block == 128)
    return launch4q<128, false, true, false>(s, rays, idx, n_max, count_dev, hits, refill, stats, st);
  if (!STATS && !ANY && s.quantised && block == 512)
    return launch4q<512, false, true, false>(s, rays, idx, n_max, count_dev, hits, refill, stats, st);
  return s.quantised ? launch4q<kTraceBlock, STATS, true, ANY>(s, rays, idx, n_max, count_dev, hits, refill, stats, st)
                     : launch4q<kTraceBlock, STATS, false, ANY>(s, rays, idx, n_max, count_dev, hits, refill, stats,
                                                                st);
}

}  // namespace

rr_status launch_trace(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                       const uint32_t* count_dev, rr_hit* hits, hipStream_t st) {
  if (n_max <= 0) return RR_OK;
  if (s.quantised && n_max <= quad_capacity())
    return launch_quad<false>(s, rays, idx, n_max, count_dev, hits, st);
  return launch4<false>(s, rays, idx, n_max, count_dev, hits, 0u, nullptr, st);
}

rr_status launch_trace_refill(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                              const uint32_t* count_dev, rr_hit* hits, uint32_t refill, hipStream_t st,
                              uint32_t block) {
  return launch4<false>(s, rays, idx, n_max, count_dev, hits, refill, nullptr, st, block);
}

rr_status launch_trace_any(const DeviceScene& s, const rr_ray* rays, const uint32_t* idx, int64_t n_max,
                           const uint32_t* count_dev, rr_hit* hits, hipStream_t st) {
  if (n_max <= 0) return RR_OK;
  if (s.quantised && n_max <= quad_capacity())
    return launch_quad<true>(s, rays, idx, n_max, count_dev, hits, st);
  return launch4<false, true>(s, rays, idx, n_max, count_dev, hits, 0u, nullptr, st);
}

void trace_warm() {
  (void)quad_capacity();
  (void)resident_blocks<kTraceBlock, false, false, false>();
  (void)resident_blocks<kTraceBlock, false, true, false>();
  (void)resident_blocks<kTraceBlock, true, false, false>();
  (void)resident_blocks<kTraceBlock, true, true, false>();
  (void)resident_blocks<kTraceBlock, false, false, true>();
  (void)resident_blocks<kTraceBlock, false, true, true>();
  (void)resident_blocks<128, false, true, false>();
  (void)resident_blocks<512, false, true, false>();
}

rr_status launch_trace_stats(const DeviceScene& s, const rr_ray* rays, int64_t n_max, rr_hit* hits,
                             uint64_t* stats_dev, hipStream_t st) {
  return launch4<true>(s, rays, nullptr, n_max, nullptr, hits, 0u,
                       reinterpret_cast<TraceStats*>(stats_dev), st);
}

}  // namespace rr
