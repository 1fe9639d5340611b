// Leaf triangular solves with the stored leaf LU factors.
//
//   trans = 0:  X(I_a, :) = U_a^{-1} L_a^{-1} P_a^T B(I_a, :)
//     (Alg. "a:gpuf" batched_LU_solve_inplace on Y_big^L: one solve per leaf
//      for all R columns of U_big at once; Alg. "a:gpus" leaf solve on x)
//   trans = 1:  X(I_a, :) = P_a L_a^{-T} U_a^{-T} B(I_a, :)   (adjoint leaf solve)
//
// One workgroup (256 threads) per (leaf, 64-column chunk).  Thread t owns
// column t % 64 of the chunk and the 16-row blocks b with b % 4 == t / 64
// (block-cyclic, so the four waves share the triangular work evenly); its
// 4 x 16 values live in registers.  Each block step solves the diagonal
// 16 x 16 triangle in the owning wave, publishes the block through LDS and
// the other waves apply the rank-16 update with FMAs whose triangular-factor
// operands are wave-uniform loads.
#include "internal.h"

namespace hodlr {

constexpr int kTsCols = 64;
constexpr int kTsThreads = 256;

template <typename T, typename S, int TRANS>
__global__ __launch_bounds__(kTsThreads) void leaf_trsm_kernel(int m_max, const int64_t* __restrict__ leaf_off,
                                                               const T* __restrict__ lu,
                                                               const int32_t* __restrict__ perm,
                                                               const T* __restrict__ udinv, const S* B,
                                                               int64_t ldb, T* X, int64_t ldx, int ncols,
                                                               int nchunks) {
  __shared__ T xs[16][kTsCols];
  const int64_t nblocks = (int64_t)gridDim.x;
  const int64_t lid = xcd_remap(blockIdx.x, nblocks);
  const int a = (int)(lid / nchunks);
  const int chunk = (int)(lid % nchunks);
  const int64_t o = leaf_off[a];
  const int m = (int)(leaf_off[a + 1] - o);
  const int tid = threadIdx.x;
  const int c = tid & (kTsCols - 1);
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = chunk * kTsCols + c;
  const bool cok = col < ncols;
  const int nbk = (m + 15) >> 4;
  const T* F = lu + (int64_t)a * m_max * m_max;  // col-major, ld = m_max, zero padded
  const int32_t* pm = perm + (int64_t)a * m_max;
  const T* ud = udinv + (int64_t)a * m_max;
  // factor entry (i, j) of the padded block (zero outside m x m)
  auto Fe = [&](int i, int j) -> T { return F[i + (int64_t)j * m_max]; };

  T x[4][16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = 4 * q + g;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 16 * b + i;
      T v = T(0);
      if (cok && row < m) {
        const int src = TRANS ? row : pm[row];
        v = (T)B[o + src + (int64_t)col * ldb];
      }
      x[q][i] = v;
    }
  }
  __syncthreads();  // B may alias X: every load of this chunk happens before any store

  // ---- first sweep (forward): L (unit lower) or U^T (lower, non-unit) ----
  for (int k = 0; k < nbk; ++k) {
    if ((k & 3) == g) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * q + g == k) {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            if (TRANS) x[q][j] *= ud[16 * k + j];
#pragma unroll
            for (int i = j + 1; i < 16; ++i) {
              const T f = TRANS ? Fe(16 * k + j, 16 * k + i) : Fe(16 * k + i, 16 * k + j);
              x[q][i] -= f * x[q][j];
            }
          }
#pragma unroll
          for (int j = 0; j < 16; ++j) xs[j][c] = x[q][j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = 4 * q + g;
      if (b > k && b < nbk) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const T xv = xs[j][c];
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const T f = TRANS ? Fe(16 * k + j, 16 * b + i) : Fe(16 * b + i, 16 * k + j);
            x[q][i] -= f * xv;
          }
        }
      }
    }
    __syncthreads();
  }
  // ---- second sweep (backward): U (upper, non-unit) or L^T (unit upper) ----
  for (int k = nbk - 1; k >= 0; --k) {
    if ((k & 3) == g) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * q + g == k) {
#pragma unroll
          for (int j = 15; j >= 0; --j) {
            if (!TRANS) x[q][j] *= ud[16 * k + j];
#pragma unroll
            for (int i = 0; i < j; ++i) {
              const T f = TRANS ? Fe(16 * k + j, 16 * k + i) : Fe(16 * k + i, 16 * k + j);
              x[q][i] -= f * x[q][j];
            }
          }
#pragma unroll
          for (int j = 0; j < 16; ++j) xs[j][c] = x[q][j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = 4 * q + g;
      if (b < k) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const T xv = xs[j][c];
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const T f = TRANS ? Fe(16 * k + j, 16 * b + i) : Fe(16 * b + i, 16 * k + j);
            x[q][i] -= f * xv;
          }
        }
      }
    }
    __syncthreads();
  }
  // ---- store (transposed solve scatters rows through the permutation) ----
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = 4 * q + g;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 16 * b + i;
      if (cok && row < m) {
        const int dst = TRANS ? pm[row] : row;
        X[o + dst + (int64_t)col * ldx] = x[q][i];
      }
    }
  }
}

template <typename T, typename S>
hipError_t launch_leaf_trsm(hipStream_t s, int trans, int nleaf, int m_max, const int64_t* d_leaf_off,
                            const T* lu, const int32_t* perm, const T* udinv, const S* B, int64_t ldb, T* X,
                            int64_t ldx, int ncols) {
  if (nleaf == 0 || ncols == 0) return hipSuccess;
  const int nchunks = (ncols + kTsCols - 1) / kTsCols;
  const int64_t grid = (int64_t)nleaf * nchunks;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (trans)
    hipLaunchKernelGGL((leaf_trsm_kernel<T, S, 1>), dim3((unsigned)grid), dim3(kTsThreads), 0, s, m_max,
                       d_leaf_off, lu, perm, udinv, B, ldb, X, ldx, ncols, nchunks);
  else
    hipLaunchKernelGGL((leaf_trsm_kernel<T, S, 0>), dim3((unsigned)grid), dim3(kTsThreads), 0, s, m_max,
                       d_leaf_off, lu, perm, udinv, B, ldb, X, ldx, ncols, nchunks);
  return hipGetLastError();
}

template hipError_t launch_leaf_trsm<double, double>(hipStream_t, int, int, int, const int64_t*, const double*,
                                                     const int32_t*, const double*, const double*, int64_t,
                                                     double*, int64_t, int);
template hipError_t launch_leaf_trsm<float, double>(hipStream_t, int, int, int, const int64_t*, const float*,
                                                    const int32_t*, const float*, const double*, int64_t,
                                                    float*, int64_t, int);
template hipError_t launch_leaf_trsm<float, float>(hipStream_t, int, int, int, const int64_t*, const float*,
                                                   const int32_t*, const float*, const float*, int64_t, float*,
                                                   int64_t, int);

}  // namespace hodlr
