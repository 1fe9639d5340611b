// MFMA helpers shared by the HIP kernels (f64 16x16x4 and f32 16x16x4).
//
// Operand layouts (wave of 64 lanes, li = lane % 16, lq = lane / 16):
//   A (16 x 4):  lane holds A[li][lq]
//   B (4 x 16):  lane holds B[lq][li]
//   C (16 x 16): register t of a lane holds C[crow(lq, t)][li], where
//                crow = 4t + lq for f64 and 4lq + t for f32 (measured on gfx950).
// Register t of an accumulator therefore holds one 4-row K-step of the tile
// (rows crow(0..3, t)); used as a B operand, the matching A operand takes
// column crow(lq, t) of the left factor.
#pragma once
#include "internal.h"

namespace hodlr {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 V;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int lq, int t) { return 4 * t + lq; }
};
template <>
struct Mfma<float> {
  typedef f4 V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int lq, int t) { return 4 * lq + t; }
};

template <typename V>
__device__ __forceinline__ V vzero() {
  V v;
  v[0] = 0;
  v[1] = 0;
  v[2] = 0;
  v[3] = 0;
  return v;
}

}  // namespace hodlr
