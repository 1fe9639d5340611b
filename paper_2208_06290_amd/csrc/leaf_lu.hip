// Batched LU with partial pivoting of the leaf diagonal blocks
// (Alg. "a:fact" leaf loop / Alg. "a:gpuf" batched_LU_factorize_inplace on D_big^L).
//
// One workgroup (256 threads) per leaf.  Right-looking blocked LU with panels
// of kNB columns: the panel is factored in LDS (pivot = largest magnitude,
// lowest row on ties, as LAPACK's idamax), row interchanges are applied to the
// rest of the block, U12 = L11^{-1} A12 is solved per column and the trailing
// block is updated from LDS-resident L21 / U12 with 4x4 register tiles.
//
// Output per leaf a (block of ldl x ldl, column-major, ld = ldl; ldl = m_max rounded up to 16):
//   lu     unit-lower L below the diagonal, U on and above; zero outside m_a x m_a
//          (the padding lets the 16-row block solves run without bounds checks)
//   piv    LAPACK-style interchanges: row j was swapped with piv[j] (0-based, >= j)
//   perm   composed row order: row i of P^T A is row perm[i] of A
//   udinv  1 / U_jj (1 outside m_a)
// First exactly-zero pivot -> atomicMin(info, leaf << 20 | column).
#include "internal.h"

namespace hodlr {

constexpr int kNB = 32;
constexpr int kLuThreads = 256;

template <typename T>
__device__ __forceinline__ void argmax_abs_wave(T& v, int& i) {
  // max |value|, lowest index on ties, across the 64 lanes of a wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T ov = __shfl_xor(v, off, 64);
    int oi = __shfl_xor(i, off, 64);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

template <typename T, typename S>
__global__ __launch_bounds__(kLuThreads) void leaf_lu_kernel(int m_max, const int64_t* __restrict__ leaf_off,
                                                             const S* __restrict__ D, int64_t ldd,
                                                             T* __restrict__ lu, int32_t* __restrict__ piv,
                                                             int32_t* __restrict__ perm, T* __restrict__ udinv,
                                                             unsigned long long* info) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Ps = reinterpret_cast<T*>(smem_raw);                 // panel: rows 0..pr-1, ld = kLeafLd
  constexpr int kLeafLd = HODLR_MAX_LEAF;
  T* Us = Ps + kLeafLd * kNB;                             // U12 block: kNB x (<= 256), row-major ld 256
  __shared__ T redv[kLuThreads / 64];
  __shared__ int redi[kLuThreads / 64];
  __shared__ int spiv[kNB];
  __shared__ T spivval;

  const int a = blockIdx.x;
  const int64_t o = leaf_off[a];
  const int m = (int)(leaf_off[a + 1] - o);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  T* A = lu + (int64_t)a * m_max * m_max;
  int32_t* pv = piv + (int64_t)a * m_max;

  // copy D_a into the factor block, zero padding outside m x m
  for (int64_t e = tid; e < (int64_t)m_max * m_max; e += kLuThreads) {
    int i = (int)(e % m_max), j = (int)(e / m_max);
    A[e] = (i < m && j < m) ? (T)D[o + i + (int64_t)j * ldd] : T(0);
  }
  __syncthreads();

  for (int k0 = 0; k0 < m; k0 += kNB) {
    const int nb = min(kNB, m - k0);
    const int pr = m - k0;  // panel rows
    for (int e = tid; e < pr * nb; e += kLuThreads) {
      int i = e % pr, j = e / pr;
      Ps[i + j * kLeafLd] = A[(k0 + i) + (int64_t)(k0 + j) * m_max];
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      // pivot search in column j, rows j..pr-1 (one candidate per thread)
      T best = T(-1);
      int bi = 0x7fffffff;
      for (int i = j + tid; i < pr; i += kLuThreads) {
        T v = fabs(Ps[i + j * kLeafLd]);
        if (v > best || (v == best && i < bi)) {
          best = v;
          bi = i;
        }
      }
      argmax_abs_wave(best, bi);
      if (lane == 0) {
        redv[wid] = best;
        redi[wid] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        T bv = redv[0];
        int bx = redi[0];
        for (int w = 1; w < kLuThreads / 64; ++w)
          if (redv[w] > bv || (redv[w] == bv && redi[w] < bx)) {
            bv = redv[w];
            bx = redi[w];
          }
        if (bx >= pr) bx = j;  // no comparable candidate (NaN column): keep the diagonal
        spiv[j] = bx;
        spivval = Ps[bx + j * kLeafLd];
        pv[k0 + j] = k0 + bx;
        if (spivval == T(0)) atomicMin(info, ((unsigned long long)a << 20) | (unsigned long long)(k0 + j));
      }
      __syncthreads();
      const int p = spiv[j];
      const T pivot = spivval;
      if (p != j)
        for (int c = tid; c < nb; c += kLuThreads) {
          T t0 = Ps[j + c * kLeafLd];
          Ps[j + c * kLeafLd] = Ps[p + c * kLeafLd];
          Ps[p + c * kLeafLd] = t0;
        }
      __syncthreads();
      if (pivot != T(0)) {
        const T rinv = T(1) / pivot;
        for (int i = j + 1 + tid; i < pr; i += kLuThreads) {
          T l = Ps[i + j * kLeafLd] * rinv;
          Ps[i + j * kLeafLd] = l;
          for (int c = j + 1; c < nb; ++c) Ps[i + c * kLeafLd] -= l * Ps[j + c * kLeafLd];
        }
      }
      __syncthreads();
    }
    // panel back to global
    for (int e = tid; e < pr * nb; e += kLuThreads) {
      int i = e % pr, j = e / pr;
      A[(k0 + i) + (int64_t)(k0 + j) * m_max] = Ps[i + j * kLeafLd];
    }
    // interchanges on the columns left and right of the panel
    for (int c = tid; c < m; c += kLuThreads) {
      if (c >= k0 && c < k0 + nb) continue;
      T* col = A + (int64_t)c * m_max;
      for (int j = 0; j < nb; ++j) {
        int p = spiv[j];
        if (p != j) {
          T t0 = col[k0 + j];
          col[k0 + j] = col[k0 + p];
          col[k0 + p] = t0;
        }
      }
    }
    __syncthreads();
    const int rest = m - k0 - nb;
    if (rest > 0) {
      // U12 = L11^{-1} A12, one column per thread
      for (int c = tid; c < rest; c += kLuThreads) {
        T* col = A + (int64_t)(k0 + nb + c) * m_max + k0;
        T x[kNB];
#pragma unroll
        for (int i = 0; i < kNB; ++i) x[i] = (i < nb) ? col[i] : T(0);
#pragma unroll
        for (int i = 1; i < kNB; ++i) {
          if (i < nb) {
            T acc = x[i];
#pragma unroll
            for (int jj = 0; jj < kNB; ++jj)
              if (jj < i) acc -= Ps[i + jj * kLeafLd] * x[jj];
            x[i] = acc;
          }
        }
#pragma unroll
        for (int i = 0; i < kNB; ++i)
          if (i < nb) {
            col[i] = x[i];
            Us[i * kLeafLd + c] = x[i];
          }
      }
      __syncthreads();
      // A22 -= L21 * U12 with 4x4 register tiles over 64x64 sub-blocks
      const int tx = tid >> 4, ty = tid & 15;
      for (int rb = 0; rb < rest; rb += 64)
        for (int cb = 0; cb < rest; cb += 64) {
          T acc[4][4];
#pragma unroll
          for (int ii = 0; ii < 4; ++ii)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              int r = rb + ty + 16 * ii, c = cb + tx + 16 * jj;
              acc[ii][jj] = (r < rest && c < rest) ? A[(k0 + nb + r) + (int64_t)(k0 + nb + c) * m_max] : T(0);
            }
          for (int kk = 0; kk < nb; ++kk) {
            T lv[4], uv[4];
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) {
              int r = rb + ty + 16 * ii;
              lv[ii] = (r < rest) ? Ps[(nb + r) + kk * kLeafLd] : T(0);
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              int c = cb + tx + 16 * jj;
              uv[jj] = (c < rest) ? Us[kk * kLeafLd + c] : T(0);
            }
#pragma unroll
            for (int ii = 0; ii < 4; ++ii)
#pragma unroll
              for (int jj = 0; jj < 4; ++jj) acc[ii][jj] -= lv[ii] * uv[jj];
          }
#pragma unroll
          for (int ii = 0; ii < 4; ++ii)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              int r = rb + ty + 16 * ii, c = cb + tx + 16 * jj;
              if (r < rest && c < rest) A[(k0 + nb + r) + (int64_t)(k0 + nb + c) * m_max] = acc[ii][jj];
            }
        }
    }
    __syncthreads();
  }
  // composed permutation and reciprocal diagonal
  int32_t* pm = perm + (int64_t)a * m_max;
  T* ud = udinv + (int64_t)a * m_max;
  for (int i = tid; i < m_max; i += kLuThreads) {
    ud[i] = (i < m) ? T(1) / A[i + (int64_t)i * m_max] : T(1);
    if (i >= m) pv[i] = i;
  }
  if (tid == 0) {
    for (int i = 0; i < m_max; ++i) pm[i] = i;
    for (int j = 0; j < m; ++j) {
      int p = pv[j];
      int t0 = pm[j];
      pm[j] = pm[p];
      pm[p] = t0;
    }
  }
}

template <typename T, typename S>
hipError_t launch_leaf_lu(hipStream_t s, int nleaf, int m_max, const int64_t* d_leaf_off, const S* D,
                          int64_t ldd, T* lu, int32_t* piv, int32_t* perm, T* udinv,
                          unsigned long long* info) {
  if (nleaf == 0) return hipSuccess;
  size_t smem = sizeof(T) * (size_t)(HODLR_MAX_LEAF * kNB * 2);
  auto k = leaf_lu_kernel<T, S>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(nleaf), dim3(kLuThreads), smem, s, m_max, d_leaf_off, D, ldd, lu, piv, perm, udinv,
                     info);
  return hipGetLastError();
}

template hipError_t launch_leaf_lu<double, double>(hipStream_t, int, int, const int64_t*, const double*, int64_t,
                                                   double*, int32_t*, int32_t*, double*, unsigned long long*);
template hipError_t launch_leaf_lu<float, double>(hipStream_t, int, int, const int64_t*, const double*, int64_t,
                                                  float*, int32_t*, int32_t*, float*, unsigned long long*);
template hipError_t launch_leaf_lu<float, float>(hipStream_t, int, int, const int64_t*, const float*, int64_t,
                                                 float*, int32_t*, int32_t*, float*, unsigned long long*);

}  // namespace hodlr
