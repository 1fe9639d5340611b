// Wave-level reductions on DPP lane moves (no LDS round trips): quad
// permutations, row mirrors and the gfx9 row broadcasts combine the 64 lanes
// in six steps; lane 63 then holds the result, which readlane makes uniform.
#pragma once
#include "internal.h"

namespace hodlr {

namespace dpp {
constexpr int kQuad1032 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int kQuad2301 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kRowBcast15 = 0x142;   // lane 15 of each row into the next row (rows 1, 3 enabled)
constexpr int kRowBcast31 = 0x143;   // lane 31 into rows 2 and 3

template <int CTRL, int ROWS>
__device__ __forceinline__ int mov(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double mov(double v) {
  int2 x = __builtin_bit_cast(int2, v);
  x.x = __builtin_amdgcn_update_dpp(x.x, x.x, CTRL, ROWS, 0xf, false);
  x.y = __builtin_amdgcn_update_dpp(x.y, x.y, CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, x);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, v), __builtin_bit_cast(int, v),
                                                               CTRL, ROWS, 0xf, false));
}
__device__ __forceinline__ int uniform63(int v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ __forceinline__ double uniform63(double v) {
  int2 x = __builtin_bit_cast(int2, v);
  x.x = __builtin_amdgcn_readlane(x.x, 63);
  x.y = __builtin_amdgcn_readlane(x.y, 63);
  return __builtin_bit_cast(double, x);
}
__device__ __forceinline__ float uniform63(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
}  // namespace dpp

// maximum over the wave (NaN-free inputs), uniform result
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  v = max(v, dpp::mov<dpp::kQuad1032, 0xf>(v));
  v = max(v, dpp::mov<dpp::kQuad2301, 0xf>(v));
  v = max(v, dpp::mov<dpp::kRowHalfMirror, 0xf>(v));
  v = max(v, dpp::mov<dpp::kRowMirror, 0xf>(v));
  v = max(v, dpp::mov<dpp::kRowBcast15, 0xa>(v));
  v = max(v, dpp::mov<dpp::kRowBcast31, 0xc>(v));
  return dpp::uniform63(v);
}
__device__ __forceinline__ int wave_min(int v) {
  v = min(v, dpp::mov<dpp::kQuad1032, 0xf>(v));
  v = min(v, dpp::mov<dpp::kQuad2301, 0xf>(v));
  v = min(v, dpp::mov<dpp::kRowHalfMirror, 0xf>(v));
  v = min(v, dpp::mov<dpp::kRowMirror, 0xf>(v));
  v = min(v, dpp::mov<dpp::kRowBcast15, 0xa>(v));
  v = min(v, dpp::mov<dpp::kRowBcast31, 0xc>(v));
  return dpp::uniform63(v);
}

// Pivot search: the largest v over the wave and, among the lanes holding it,
// the smallest key (v >= 0 for candidates, -1 otherwise; NaN mapped to
// infinity by the caller).  Both results are uniform.
template <typename T>
__device__ __forceinline__ void wave_argmax(T v, int key, T& vmax, int& kmin) {
  vmax = wave_max(v);
  const unsigned long long hit = __ballot(v == vmax);
  if (__builtin_popcountll(hit) == 1)
    kmin = __builtin_amdgcn_readlane(key, (int)__builtin_ctzll(hit));
  else
    kmin = wave_min(v == vmax ? key : 0x7fffffff);
}

}  // namespace hodlr
