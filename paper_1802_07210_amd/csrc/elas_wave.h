// Wavefront-wide operations without LDS: DPP exchanges within 16-lane rows
// (quad permutes, the half-row and row mirrors, row shifts) and lane reads
// across the four rows. Every function here needs all 64 lanes of the
// wavefront active (the quad exchanges: all four lanes of the quad); the
// callers run them in wavefront-uniform control flow.
#ifndef ELAS_WAVE_H
#define ELAS_WAVE_H

#include <hip/hip_runtime.h>

#include <cstdint>

namespace elas {

// DPP controls: quad permutes [1,0,3,2] and [2,3,0,1], row mirrors, row shifts
constexpr int kDppQuadXor1 = 0xB1;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowShr1 = 0x111;

// Lane i of the quad gets lane i ^ 1 / i ^ 2 of the same quad.
__device__ __forceinline__ int quad_xor1(int x) {
  return __builtin_amdgcn_update_dpp(x, x, kDppQuadXor1, 0xF, 0xF, false);
}
__device__ __forceinline__ int quad_xor2(int x) {
  return __builtin_amdgcn_update_dpp(x, x, kDppQuadXor2, 0xF, 0xF, false);
}

// Every lane of a row ends with the row's minimum / sum.
__device__ __forceinline__ uint32_t row_min_u32(uint32_t x) {
  x = min(x, (uint32_t)quad_xor1((int)x));
  x = min(x, (uint32_t)quad_xor2((int)x));
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, kDppRowHalfMirror, 0xF, 0xF,
                                                     false));
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, kDppRowMirror, 0xF, 0xF,
                                                     false));
  return x;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  x = row_min_u32(x);
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 0);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 16);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 32);
  const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
  return min(min(r0, r1), min(r2, r3));
}

__device__ __forceinline__ int wave_sum_i32(int x) {
  x += quad_xor1(x);
  x += quad_xor2(x);
  x += __builtin_amdgcn_update_dpp(x, x, kDppRowHalfMirror, 0xF, 0xF, false);
  x += __builtin_amdgcn_update_dpp(x, x, kDppRowMirror, 0xF, 0xF, false);
  return __builtin_amdgcn_readlane(x, 0) + __builtin_amdgcn_readlane(x, 16) +
         __builtin_amdgcn_readlane(x, 32) + __builtin_amdgcn_readlane(x, 48);
}

// 64-bit minimum: both halves take the same exchange, then one comparison.
template <int kCtl>
__device__ __forceinline__ unsigned long long min_dpp_u64(unsigned long long v) {
  const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  const int olo = __builtin_amdgcn_update_dpp(lo, lo, kCtl, 0xF, 0xF, false);
  const int ohi = __builtin_amdgcn_update_dpp(hi, hi, kCtl, 0xF, 0xF, false);
  const unsigned long long o = ((unsigned long long)(uint32_t)ohi << 32) | (uint32_t)olo;
  return o < v ? o : v;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  v = min_dpp_u64<kDppQuadXor1>(v);
  v = min_dpp_u64<kDppQuadXor2>(v);
  v = min_dpp_u64<kDppRowHalfMirror>(v);
  v = min_dpp_u64<kDppRowMirror>(v);
  unsigned long long r = ~0ull;
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const unsigned long long lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 16 * row);
    const unsigned long long hi =
        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 16 * row);
    const unsigned long long o = (hi << 32) | lo;
    r = o < r ? o : r;
  }
  return r;
}

// Inclusive prefix sum over the lanes: Hillis-Steele within each row by row
// shifts of 1, 2, 4 and 8 (a missing source reads 0), then the totals of the
// earlier rows.
__device__ __forceinline__ int wave_scan_incl(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr1, 0xF, 0xF, true);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr1 + 1, 0xF, 0xF, true);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr1 + 3, 0xF, 0xF, true);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr1 + 7, 0xF, 0xF, true);
  const int lane = threadIdx.x & 63;
  const int s0 = __builtin_amdgcn_readlane(x, 15), s1 = __builtin_amdgcn_readlane(x, 31),
            s2 = __builtin_amdgcn_readlane(x, 47);
  return x + (lane >= 16 ? s0 : 0) + (lane >= 32 ? s1 : 0) + (lane >= 48 ? s2 : 0);
}

}  // namespace elas

#endif  // ELAS_WAVE_H
