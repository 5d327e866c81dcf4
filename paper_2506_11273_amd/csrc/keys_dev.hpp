// Device-side sort-key arithmetic shared by the per-call and batched key
// kernels (Section 3.1, Figure "codes"): quantisation of a coordinate to b
// bits and placement of its bits into the key at a fixed stride.
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

template <int KIND>
__device__ __forceinline__ uint64_t ray_key(const float4 a, const float4 b, const KeyPlan& P) {
  // a = (org.xyz, tmin), b = (dir.xyz, tmax)
  const uint32_t qx = quantize(a.x, P.lo[0], P.inv[0], P.scale[0], P.qmax[0]);
  const uint32_t qy = quantize(a.y, P.lo[1], P.inv[1], P.scale[1], P.qmax[1]);
  const uint32_t qz = quantize(a.z, P.lo[2], P.inv[2], P.scale[2], P.qmax[2]);
  if constexpr (KIND == RR_KEY_ORIGIN_DIRECTION) {
    const uint32_t dx = quantize(b.x, -1.0f, 0.5f, P.scale[3], P.qmax[3]);
    const uint32_t dy = quantize(b.y, -1.0f, 0.5f, P.scale[4], P.qmax[4]);
    const uint32_t dz = quantize(b.z, -1.0f, 0.5f, P.scale[5], P.qmax[5]);
    return (spread3(qx) << P.shift[0]) | (spread3(qy) << P.shift[1]) | (spread3(qz) << P.shift[2]) |
           (spread3(dx) << P.shift[3]) | (spread3(dy) << P.shift[4]) | (spread3(dz) << P.shift[5]);
  } else {
    const float len = (b.w < P.len) ? b.w : P.len;
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
}

}  // namespace
}  // namespace rr
