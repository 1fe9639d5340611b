// Block triangular solves with stored LU factors, on MFMA.
//
//   trans = 0:  X = U^{-1} L^{-1} P^T B     (per block: P^T B takes rows perm[i])
//   trans = 1:  X = P L^{-T} U^{-T} B       (adjoint; rows scattered through perm)
//
// Used for the leaf solves of the factorization (Alg. "a:gpuf":
// batched_LU_solve_inplace on Y_big^L, all R columns of a leaf at once) and
// of the solution stage (Alg. "a:gpus"), and for the coupling solves with the
// LU of K (eqs. "e:node1", "e:node3").
//
// One workgroup (256 threads = 4 waves) per (block, 64-column chunk).  The
// chunk (<= 256 rows) stays in MFMA accumulators for the whole solve: wave w
// owns the 16-row blocks b with b % 4 == w.  The inverses of the 16 x 16
// diagonal blocks of L and U come with the factorization and are staged in
// LDS per sweep, so every block step is a contraction: the owning wave forms
// X_k = inv(M_kk) B_k
// (the accumulator registers of B_k are exactly the B operands of that
// product), publishes X_k through LDS (double buffered, one barrier per
// step), and every wave applies B_b -= M_bk X_k to its blocks on MFMA with
// operands fetched before the barrier.
#include "mfma.h"

namespace hodlr {

constexpr int kTsThreads = 256;

template <typename T, typename S, int TRANS>
__global__ __launch_bounds__(kTsThreads, 2) void trsm_kernel(int ldl, const int64_t* __restrict__ leaf_off,
                                                             int64_t ostride, int mfix, const T* __restrict__ lu,
                                                             const int32_t* __restrict__ perm,
                                                             const T* __restrict__ dinv, const S* B, int64_t ldb,
                                                             T* X, int64_t ldx, int ncols, int nchunks) {
  using M = Mfma<T>;
  using V = typename M::V;
  __shared__ T invA[16 * 256];     // inverse diagonal blocks of the current sweep, [kb][i][j]
  __shared__ T xk[2][16 * 64];     // published block X_k: [row][col]

  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  const int a = (int)(lid / nchunks);
  const int chunk = (int)(lid % nchunks);
  int64_t o;
  int m;
  if (leaf_off) {
    o = leaf_off[a];
    m = (int)(leaf_off[a + 1] - o);
  } else {
    o = (int64_t)a * ostride;
    m = mfix;
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lq = lane >> 4;
  const int c0 = chunk * 64;
  const int ncb = min(4, (ncols - c0 + 15) >> 4);
  const int nbk = (m + 15) >> 4;
  const T* F = lu + (int64_t)a * ldl * ldl;
  const int32_t* pm = perm + (int64_t)a * ldl;
  const int nbd = ldl >> 4;
  const T* DI = dinv + (int64_t)a * 2 * nbd * 256;  // [0][kb]: inv(L_kk), [1][kb]: inv(U_kk)

  // F(i, j) of the zero-padded factor block; U's padded diagonal reads as 1
  auto Fe = [&](int i, int j) -> T { return F[i + (int64_t)j * ldl]; };
  auto Ud = [&](int i) -> T { return i < m ? F[i + (int64_t)i * ldl] : T(1); };
  // sweep matrix element (global indices): sweep 0 is lower, sweep 1 upper
  auto Mel = [&](int sweep, int i, int j) -> T {
    if (!TRANS) {
      if (sweep == 0) return i == j ? T(1) : (i > j ? Fe(i, j) : T(0));   // L
      return i == j ? Ud(i) : (i < j ? Fe(i, j) : T(0));                  // U
    } else {
      if (sweep == 0) return i == j ? Ud(i) : (i > j ? Fe(j, i) : T(0));  // U^T
      return i == j ? T(1) : (i < j ? Fe(j, i) : T(0));                   // L^T
    }
  };
  // stage inv(M_kk) of a sweep: sweep 0 is L (trans 0) or U^T (trans 1), sweep 1 is U or L^T
  auto stage_inv = [&](int sweep) {
    const int which = TRANS ? 1 - sweep : sweep;
    const T* src = DI + (int64_t)which * nbd * 256;
    for (int e = tid; e < nbk * 256; e += kTsThreads) {
      const int kb = e >> 8, i = (e >> 4) & 15, j = e & 15;
      invA[e] = TRANS ? src[kb * 256 + j * 16 + i] : src[e];
    }
  };

  stage_inv(0);

  // load the chunk (rows of P^T B for trans = 0) into accumulators
  V acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = 16 * (4 * q + w) + M::crow(lq, t);
        const int col = c0 + 16 * cb + li;
        T v = T(0);
        if (cb < ncb && row < m && col < ncols) {
          const int src = TRANS ? row : pm[row];
          v = (T)B[o + src + (int64_t)col * ldb];
        }
        acc[q][cb][t] = v;
      }
  __syncthreads();  // invA staged; B may alias X: all loads of the chunk precede any store

#pragma unroll
  for (int sweep = 0; sweep < 2; ++sweep) {
    if (sweep == 1) {
      __syncthreads();
      stage_inv(1);
      __syncthreads();
    }
    for (int step = 0; step < nbk; ++step) {
      const int k = sweep == 0 ? step : nbk - 1 - step;
      T* xb = xk[step & 1];
      if ((k & 3) == w) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (4 * q + w == k) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
              if (cb < ncb) {
                V nv = vzero<V>();
#pragma unroll
                for (int t = 0; t < 4; ++t)
                  nv = M::mma(invA[k * 256 + li * 16 + M::crow(lq, t)], acc[q][cb][t], nv);
                acc[q][cb] = nv;
#pragma unroll
                for (int t = 0; t < 4; ++t) xb[M::crow(lq, t) * 64 + 16 * cb + li] = nv[t];
              }
          }
      }
      // B_b -= M_bk X_k for this wave's blocks on the far side of k; the factor
      // operands do not depend on X_k and are fetched before the barrier
      T av[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = 4 * q + w;
        const bool act = sweep == 0 ? (b > k && b < nbk) : (b < k);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) av[q][ks] = act ? -Mel(sweep, 16 * b + li, 16 * k + 4 * ks + lq) : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = 4 * q + w;
        const bool act = sweep == 0 ? (b > k && b < nbk) : (b < k);
        if (act) {
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
              if (cb < ncb) acc[q][cb] = M::mma(av[q][ks], xb[(4 * ks + lq) * 64 + 16 * cb + li], acc[q][cb]);
        }
      }
    }
  }

  // store (the adjoint scatters rows through the permutation)
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = 16 * (4 * q + w) + M::crow(lq, t);
        const int col = c0 + 16 * cb + li;
        if (cb < ncb && row < m && col < ncols) {
          const int dst = TRANS ? pm[row] : row;
          X[o + dst + (int64_t)col * ldx] = acc[q][cb][t];
        }
      }
}

template <typename T, typename S>
static hipError_t launch_trsm(hipStream_t s, int trans, int nblk, int ldl, const int64_t* d_off, int64_t ostride,
                              int mfix, const T* lu, const int32_t* perm, const T* dinv, const S* B, int64_t ldb, T* X,
                              int64_t ldx, int ncols) {
  if (nblk == 0 || ncols == 0) return hipSuccess;
  if (ldl % 16 || ldl > 256) return hipErrorInvalidValue;
  const int nchunks = (ncols + 63) / 64;
  const int64_t grid = (int64_t)nblk * nchunks;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (trans)
    hipLaunchKernelGGL((trsm_kernel<T, S, 1>), dim3((unsigned)grid), dim3(kTsThreads), 0, s, ldl, d_off, ostride,
                       mfix, lu, perm, dinv, B, ldb, X, ldx, ncols, nchunks);
  else
    hipLaunchKernelGGL((trsm_kernel<T, S, 0>), dim3((unsigned)grid), dim3(kTsThreads), 0, s, ldl, d_off, ostride,
                       mfix, lu, perm, dinv, B, ldb, X, ldx, ncols, nchunks);
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_leaf_trsm(hipStream_t s, int trans, int nleaf, int ldl, const int64_t* d_leaf_off, const T* lu,
                            const int32_t* perm, const T* dinv, const S* B, int64_t ldb, T* X, int64_t ldx,
                            int ncols) {
  return launch_trsm<T, S>(s, trans, nleaf, ldl, d_leaf_off, 0, 0, lu, perm, dinv, B, ldb, X, ldx, ncols);
}

template <typename T>
hipError_t launch_block_trsm(hipStream_t s, int trans, int nblk, int ldl, int m, int64_t ostride, const T* lu,
                             const int32_t* perm, const T* dinv, T* X, int64_t ldx, int ncols) {
  return launch_trsm<T, T>(s, trans, nblk, ldl, nullptr, ostride, m, lu, perm, dinv, X, ldx, X, ldx, ncols);
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
template hipError_t launch_block_trsm<double>(hipStream_t, int, int, int, int, int64_t, const double*,
                                              const int32_t*, const double*, double*, int64_t, int);
template hipError_t launch_block_trsm<float>(hipStream_t, int, int, int, int, int64_t, const float*, const int32_t*,
                                             const float*, float*, int64_t, int);

}  // namespace hodlr
