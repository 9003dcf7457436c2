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

// DPP row broadcasts: lane 15 of each row to the next row, lane 31 to rows
// 2 and 3.
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

// The value of lane ctl(i) for a control under which every lane has a valid
// source (quad permutes, mirrors). The form (old 0, bound_ctrl) lets the
// compiler fold the exchange into the DPP operand of the ALU op that uses it.
template <int kCtl>
__device__ __forceinline__ uint32_t dpp_full(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kCtl, 0xF, 0xF, true);
}

// Every lane of a row ends with the row's minimum / sum.
__device__ __forceinline__ uint32_t row_min_u32(uint32_t x) {
  x = min(x, dpp_full<kDppQuadXor1>(x));
  x = min(x, dpp_full<kDppQuadXor2>(x));
  x = min(x, dpp_full<kDppRowHalfMirror>(x));
  return min(x, dpp_full<kDppRowMirror>(x));
}

__device__ __forceinline__ uint32_t row_sum_u32(uint32_t x) {
  x += dpp_full<kDppQuadXor1>(x);
  x += dpp_full<kDppQuadXor2>(x);
  x += dpp_full<kDppRowHalfMirror>(x);
  return x + dpp_full<kDppRowMirror>(x);
}

// Row results to lane 63: row 1 takes row 0's and row 3 row 2's (lane 15 of
// the row before), then rows 2 and 3 take row 1's (lane 31). Rows outside a
// broadcast's row mask get the operation's identity.
__device__ __forceinline__ uint32_t rows_min_to_lane63(uint32_t x) {
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, kDppRowBcast15, 0xA, 0xF, false));
  return min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, kDppRowBcast31, 0xC, 0xF, false));
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readlane((int)rows_min_to_lane63(row_min_u32(x)), 63);
}

__device__ __forceinline__ int wave_sum_i32(int x) {
  uint32_t y = row_sum_u32((uint32_t)x);
  y += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)y, kDppRowBcast15, 0xA, 0xF, false);
  y += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)y, kDppRowBcast31, 0xC, 0xF, false);
  return __builtin_amdgcn_readlane((int)y, 63);
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
