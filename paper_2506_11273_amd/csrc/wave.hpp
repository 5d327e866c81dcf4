// Wave64 helpers of the radix sorts (device code only).
#pragma once

#include "common.hpp"

namespace rr {
namespace {

// Number of lanes of m below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes among `valid` whose DB-bit digit equals this lane's d: one ballot
// per bit, each lane keeping the lanes that agree with it on that bit.
// bitop3 with table 0x84 computes b & ~(a ^ c) (only the input patterns
// (0,1,0) and (1,1,1) give 1, the same under either operand order), with the
// ballot word as a, the running mask as b and the bit spread to a
// 0 / all-ones word as c: four VALU instructions per bit.
template <int DB>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
  uint32_t lo = (uint32_t)valid, hi = (uint32_t)(valid >> 32);
#pragma unroll
  for (int b = 0; b < DB; ++b) {
    uint32_t c = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
    asm("" : "+v"(c));  // keeps the ballot on this word (one compare) instead of a re-derived shift
    const uint64_t m = __ballot(c != 0u);
    lo = __builtin_amdgcn_bitop3_b32((uint32_t)m, lo, c, 0x84);
    hi = __builtin_amdgcn_bitop3_b32((uint32_t)(m >> 32), hi, c, 0x84);
  }
  return ((uint64_t)hi << 32) | lo;
}

}  // namespace
}  // namespace rr
