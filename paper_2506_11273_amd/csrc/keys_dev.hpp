// Device-side sort-key arithmetic shared by the per-call and batched key
// kernels (Section 3.1, Figure "codes"): quantisation of a coordinate to b
// bits, placement of its bits into the key at a fixed stride, the
// termination estimates of Section 3.1.6 and the octahedral direction.
#pragma once

#include "common.hpp"

#pragma clang fp contract(off)

namespace rr {
namespace {

// bit i of x (i < 21) -> bit 3i
__device__ __forceinline__ uint64_t spread3(uint64_t x) {
  x &= 0x1FFFFFull;
  x = (x | (x << 32)) & 0x001F00000000FFFFull;
  x = (x | (x << 16)) & 0x001F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// bit i of x (i < 16) -> bit 2i
__device__ __forceinline__ uint64_t spread2(uint64_t x) {
  x &= 0xFFFFull;
  x = (x | (x << 8)) & 0x00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0Full;
  x = (x | (x << 2)) & 0x33333333ull;
  x = (x | (x << 1)) & 0x55555555ull;
  return x;
}

__device__ __forceinline__ uint32_t quantize(float x, float lo, float inv, float scale, uint32_t qmax) {
  float u = (x - lo) * inv;
  u = (u > 0.0f) ? u : 0.0f;  // also maps NaN to 0
  u = (u > 1.0f) ? 1.0f : u;
  uint32_t q = (uint32_t)(u * scale);  // exact scaling, truncation
  return q < qmax ? q : qmax;
}

// Two Point key (Section 3.1.5): the 6-cycle interleave of origin and the
// termination point o + len * d.
__device__ __forceinline__ uint64_t two_point_key(const float4 a, const float4 b, const KeyPlan& P, float len) {
  const uint32_t qx = quantize(a.x, P.lo[0], P.inv[0], P.scale[0], P.qmax[0]);
  const uint32_t qy = quantize(a.y, P.lo[1], P.inv[1], P.scale[1], P.qmax[1]);
  const uint32_t qz = quantize(a.z, P.lo[2], P.inv[2], P.scale[2], P.qmax[2]);
  const float sx = len * b.x, sy = len * b.y, sz = len * b.z;
  const float tx = a.x + sx, ty = a.y + sy, tz = a.z + sz;
  const uint32_t ux = quantize(tx, P.lo[0], P.inv[0], P.scale[3], P.qmax[3]);
  const uint32_t uy = quantize(ty, P.lo[1], P.inv[1], P.scale[4], P.qmax[4]);
  const uint32_t uz = quantize(tz, P.lo[2], P.inv[2], P.scale[5], P.qmax[5]);
  // stride 6 = spread by 2, then by 3
  return (spread3(spread2(qx)) << P.shift[0]) | (spread3(spread2(qy)) << P.shift[1]) |
         (spread3(spread2(qz)) << P.shift[2]) | (spread3(spread2(ux)) << P.shift[3]) |
         (spread3(spread2(uy)) << P.shift[4]) | (spread3(spread2(uz)) << P.shift[5]);
}

// 20-bit length-table cell of a ray: the 20 leading slots of the Aila
// Compact layout, o12 d3 o3 d2, i.e. origin 5/5/5 bits at slots
// (19 16 13 10 4), (18 15 12 9 3), (17 14 11 8 2) and direction 2/2/1 bits
// at (7 1), (6 0), (5).
__device__ __forceinline__ uint32_t cell_code(const float4 a, const float4 b, const KeyPlan& P) {
  const uint32_t ox = quantize(a.x, P.lo[0], P.inv[0], 32.0f, 31u);
  const uint32_t oy = quantize(a.y, P.lo[1], P.inv[1], 32.0f, 31u);
  const uint32_t oz = quantize(a.z, P.lo[2], P.inv[2], 32.0f, 31u);
  const uint32_t dx = quantize(b.x, -1.0f, 0.5f, 4.0f, 3u);
  const uint32_t dy = quantize(b.y, -1.0f, 0.5f, 4.0f, 3u);
  const uint32_t dz = quantize(b.z, -1.0f, 0.5f, 2.0f, 1u);
  return ((uint32_t)spread3(ox >> 1) << 10) | ((ox & 1u) << 4) | ((uint32_t)spread3(oy >> 1) << 9) |
         ((oy & 1u) << 3) | ((uint32_t)spread3(oz >> 1) << 8) | ((oz & 1u) << 2) | ((dx >> 1) << 7) |
         ((dx & 1u) << 1) | ((dy >> 1) << 6) | (dy & 1u) | (dz << 5);
}

// Mean length of a table cell (the estimate of Two Point Adaptive).
__device__ __forceinline__ float cell_length(const rr_length_cell* T, uint32_t cell, float E) {
  const rr_length_cell c = T[cell];
  const double num = (double)c.sum * (double)E;
  const double den = (double)c.count * 16777216.0;
  return (float)(num / den);
}

// Termination length of the Two Point kinds for ray i: the fixed estimate
// (2), the table's estimate (8) or the traced hit (9, the fixed estimate
// for a miss), the estimates capped at tmax.
__device__ __forceinline__ float two_point_length(const float4 a, const float4 b, const KeyPlan& P, uint32_t i) {
  float L = P.len;
  if (P.kind == RR_KEY_TWO_POINT_ADAPTIVE)
    L = cell_length(reinterpret_cast<const rr_length_cell*>(P.aux), cell_code(a, b, P), P.E);
  float len = (b.w < L) ? b.w : L;
  if (P.kind == RR_KEY_TWO_POINT_REAL) {
    const float2 h = reinterpret_cast<const float2*>(P.aux)[2 * (size_t)i];  // (t, prim bits)
    if (__float_as_int(h.y) >= 0) len = h.x;
  }
  return len;
}

// Octahedral coordinates of a direction (Section 3.1.4, Meyer et al. 2010):
// (x, y) of d / (|d.x| + |d.y| + |d.z|), the lower half folded over the
// diagonals; sgn(0) = +1.
__device__ __forceinline__ void octahedral(float dx, float dy, float dz, float* u, float* v) {
  const float s = (fabsf(dx) + fabsf(dy)) + fabsf(dz);
  float px = dx / s;
  float py = dy / s;
  if (dz < 0.0f) {
    const float sx = px >= 0.0f ? 1.0f : -1.0f;
    const float sy = py >= 0.0f ? 1.0f : -1.0f;
    const float fx = (1.0f - fabsf(py)) * sx;
    const float fy = (1.0f - fabsf(px)) * sy;
    px = fx;
    py = fy;
  }
  *u = px;
  *v = py;
}

// bit i of x (i < cnt) -> bit stride * i
__device__ __forceinline__ uint64_t spread_by(uint32_t x, uint32_t cnt, uint32_t stride) {
  uint64_t out = 0;
  for (uint32_t i = 0; i < cnt; ++i) out |= (uint64_t)((x >> i) & 1u) << (stride * i);
  return out;
}

// The figure's other layouts, assembled field by field.
__device__ __forceinline__ uint64_t general_key(const float4 a, const float4 b, const KeyPlan& P) {
  const uint32_t q0 = quantize(a.x, P.lo[0], P.inv[0], P.scale[0], P.qmax[0]);
  const uint32_t q1 = quantize(a.y, P.lo[1], P.inv[1], P.scale[1], P.qmax[1]);
  const uint32_t q2 = quantize(a.z, P.lo[2], P.inv[2], P.scale[2], P.qmax[2]);
  uint32_t q3, q4, q5;
  if (P.kind == RR_KEY_OCTAHEDRON) {
    float u, v;
    octahedral(b.x, b.y, b.z, &u, &v);
    q3 = quantize(u, -1.0f, 0.5f, P.scale[3], P.qmax[3]);
    q4 = quantize(v, -1.0f, 0.5f, P.scale[4], P.qmax[4]);
    q5 = 0;
  } else {
    q3 = quantize(b.x, -1.0f, 0.5f, P.scale[3], P.qmax[3]);
    q4 = quantize(b.y, -1.0f, 0.5f, P.scale[4], P.qmax[4]);
    q5 = quantize(b.z, -1.0f, 0.5f, P.scale[5], P.qmax[5]);
  }
  uint64_t key = 0;
#pragma unroll
  for (int f = 0; f < kMaxKeyFields; ++f) {
    if (f >= P.nfields) break;
    const KeyField F = P.field[f];
    const uint32_t q = F.comp == 0 ? q0 : F.comp == 1 ? q1 : F.comp == 2 ? q2 : F.comp == 3 ? q3 : F.comp == 4 ? q4 : q5;
    const uint32_t bits = (q >> F.src_shift) & ((1u << F.cnt) - 1u);
    key |= spread_by(bits, F.cnt, F.stride) << F.dst_shift;
  }
  return key;
}

// Key of ray i.  KIND: 1 origin-direction, 2 the Two Point kinds, 3 the
// general layouts (the host picks it from the plan's kind).
template <int KIND>
__device__ __forceinline__ uint64_t ray_key(const float4 a, const float4 b, const KeyPlan& P, uint32_t i) {
  // a = (org.xyz, tmin), b = (dir.xyz, tmax)
  if constexpr (KIND == 1) {
    const uint32_t qx = quantize(a.x, P.lo[0], P.inv[0], P.scale[0], P.qmax[0]);
    const uint32_t qy = quantize(a.y, P.lo[1], P.inv[1], P.scale[1], P.qmax[1]);
    const uint32_t qz = quantize(a.z, P.lo[2], P.inv[2], P.scale[2], P.qmax[2]);
    const uint32_t dx = quantize(b.x, -1.0f, 0.5f, P.scale[3], P.qmax[3]);
    const uint32_t dy = quantize(b.y, -1.0f, 0.5f, P.scale[4], P.qmax[4]);
    const uint32_t dz = quantize(b.z, -1.0f, 0.5f, P.scale[5], P.qmax[5]);
    return (spread3(qx) << P.shift[0]) | (spread3(qy) << P.shift[1]) | (spread3(qz) << P.shift[2]) |
           (spread3(dx) << P.shift[3]) | (spread3(dy) << P.shift[4]) | (spread3(dz) << P.shift[5]);
  } else if constexpr (KIND == 2) {
    return two_point_key(a, b, P, two_point_length(a, b, P, i));
  } else {
    return general_key(a, b, P);
  }
}

// Template family of a key kind.
__host__ __device__ inline int key_family(int kind) {
  return kind == RR_KEY_ORIGIN_DIRECTION ? 1
         : (kind == RR_KEY_ORIGIN_TERMINATION || kind == RR_KEY_TWO_POINT_ADAPTIVE ||
            kind == RR_KEY_TWO_POINT_REAL)
             ? 2
             : 3;
}

// Key of any kind, chosen at run time (the batched kernel mixes kinds).
__device__ __forceinline__ uint64_t ray_key_any(const float4 a, const float4 b, const KeyPlan& P, uint32_t i) {
  const int f = key_family(P.kind);
  if (f == 1) return ray_key<1>(a, b, P, i);
  if (f == 2) return ray_key<2>(a, b, P, i);
  return ray_key<3>(a, b, P, i);
}

}  // namespace
}  // namespace rr
