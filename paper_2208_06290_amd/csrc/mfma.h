// MFMA helpers shared by the HIP kernels (f64 16x16x4, f32 16x16x4 and
// bf16 16x16x16 with FP32 accumulation).
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
  // crow split into a lane-uniform part (by t) and a per-lane part (by lq)
  static __device__ __forceinline__ constexpr int crow_u(int t) { return 4 * t; }
  static __device__ __forceinline__ int crow_l(int lq) { return lq; }
};
template <>
struct Mfma<float> {
  typedef f4 V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int lq, int t) { return 4 * lq + t; }
  static __device__ __forceinline__ constexpr int crow_u(int t) { return t; }
  static __device__ __forceinline__ int crow_l(int lq) { return 4 * lq; }
};

// Four 16x16x4 K-steps into one accumulator, c += sum_s (step s), where step s
// takes a[s] as the lane's A value and b[s] as its B value (whatever K index
// each step stands for).  BF = false issues the four steps in order.  BF = true
// rounds the operands to bfloat16 (nearest, ties to even) and issues one
// 16x16x16 bf16 MFMA with FP32 accumulation: that instruction takes four K
// values per lane, and a lane's four A values meet the same lane's four B
// values (element j of lane (li, lq) is K index 4 lq + j on both sides), so
// packing step s as element j = s pairs every A value with the B value of its
// own step and the sum over K is that of the four steps.
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));
template <typename T, bool BF>
struct Mma16 {
  typedef typename Mfma<T>::V V;
  static __device__ __forceinline__ V mma(const T (&a)[4], const T (&b)[4], V c) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) c = Mfma<T>::mma(a[ks], b[ks], c);
    return c;
  }
};
template <>
struct Mma16<float, true> {
  typedef f4 V;
  static __device__ __forceinline__ V mma(const float (&a)[4], const float (&b)[4], V c) {
    b4 av, bv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      av[j] = (__bf16)a[j];
      bv[j] = (__bf16)b[j];
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, av), __builtin_bit_cast(s4, bv), c, 0, 0,
                                                      0);
  }
};

// bfloat16 operands packed once (round to nearest even, as the conversions
// in Mma16<float, true>) and the 16 x 16 x 16 product on packed operands.
__device__ __forceinline__ s4 pack_bf16(const float (&x)[4]) {
  b4 v;
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = (__bf16)x[j];
  return __builtin_bit_cast(s4, v);
}
__device__ __forceinline__ f4 mma_bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Raw buffer access: a lane-uniform base in a buffer resource (scalar
// registers), a 32-bit per-lane offset and a 32-bit lane-uniform offset.
// Offsets are in bytes; callers keep every offset below 2^31.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, -1, 0x00020000);
}
template <typename T>
struct Buf;
template <>
struct Buf<double> {
  static __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, 0));
  }
  static __device__ __forceinline__ void store(double x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, x), r, (int)v, (int)s, 0);
  }
};
template <>
struct Buf<float> {
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, 0));
  }
  static __device__ __forceinline__ void store(float x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, (int)v, (int)s, 0);
  }
};

// Two consecutive elements per lane (one 8- or 16-byte access).
template <typename T>
struct Buf2;
template <>
struct Buf2<float> {
  typedef float P __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, float& x0, float& x1) {
    const P p = __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, 0));
    x0 = p[0];
    x1 = p[1];
  }
  static __device__ __forceinline__ void store(float x0, float x1, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    P p;
    p[0] = x0;
    p[1] = x1;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, p), r, (int)v, (int)s, 0);
  }
};
template <>
struct Buf2<double> {
  typedef double P __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, double& x0,
                                              double& x1) {
    const P p = __builtin_bit_cast(P, __builtin_amdgcn_raw_buffer_load_b128(r, (int)v, (int)s, 0));
    x0 = p[0];
    x1 = p[1];
  }
  static __device__ __forceinline__ void store(double x0, double x1, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                               uint32_t s) {
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    P p;
    p[0] = x0;
    p[1] = x1;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, p), r, (int)v, (int)s, 0);
  }
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
