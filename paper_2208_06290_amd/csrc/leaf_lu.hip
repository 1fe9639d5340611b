// Batched LU with partial pivoting of the leaf diagonal blocks
// (Alg. "a:fact" leaf loop / Alg. "a:gpuf" batched_LU_factorize_inplace on D_big^L).
//
// One workgroup (256 threads = 4 waves) per leaf, left-looking by 32-column
// chunks:
//   1. the chunk's original columns are loaded into MFMA accumulators in the
//      current row order (wave w owns the 16-row blocks b with b % 4 == w);
//   2. the chunk is swept with the L blocks of all earlier chunks on MFMA
//      (X_k = inv(L_kk) B_k by the owning wave, published through LDS,
//      B_b -= L_bk X_k by every wave), which leaves the U rows above the panel
//      and the Schur-complemented panel below;
//   3. the panel (rows below, 32 columns) is factored with one thread per row,
//      the row held in registers: pivot = largest magnitude, lowest current
//      position on ties (LAPACK idamax), rows are not moved - each thread
//      tracks its position; each wave publishes its best candidate's row in
//      LDS and every thread selects the winner, one barrier per column.
// Entries are stored by original row while factoring (later interchanges move
// no data); a final pass writes them in pivoted order.  Four workgroups per CU
// in FP64, five with 4-byte elements (the panel steps are latency-bound): at
// most 128 registers per lane and 40 KB of LDS, so the panel rows reach the
// registers 8 columns at a time
// and the diagonal-block inverses are formed with rolled loops, their
// columns in LDS.
//
// Output per leaf a (block of ldl x ldl, column-major, ld = ldl; ldl = m_max
// rounded up to 16; or, in place, the leaf's own rows of D with ld = ldd,
// which needs |I_a| % 16 == 0 so no 16 x 16 block reaches past the leaf):
//   lu     unit-lower L below the diagonal, U on and above; zero outside m_a x m_a
//          (the separate layout only)
//   piv    LAPACK-style interchanges: row j was swapped with piv[j] (0-based, >= j)
//   perm   composed row order: row i of P^T A is row perm[i] of A
//   udinv  1 / U_jj (1 outside m_a)
//   inv    inverses of the 16 x 16 diagonal blocks: [0][kb] = inv(L_kb,kb) (unit
//          lower), [1][kb] = inv(U_kb,kb) (upper); padded rows act as identity
// First exactly-zero pivot -> atomicMin(info, leaf << 20 | column).
#include "mfma.h"
#include "wave.h"

namespace hodlr {

constexpr int kLuThreads = 256;
constexpr int kCW = 32;  // chunk (panel) width

template <typename T, typename S, int CW, bool BF>
__global__ __launch_bounds__(kLuThreads, sizeof(T) == 4 ? 5 : 4) void leaf_lu_kernel(int ldl, const int64_t* __restrict__ leaf_off,
                                                             const S* D, int64_t ldd, T* lu, int64_t lul,
                                                             int inplace, int32_t* __restrict__ piv,
                                                             int32_t* __restrict__ perm,
                                                             T* __restrict__ udinv, T* invl,
                                                             unsigned long long* info) {
  using M = Mfma<T>;
  using V = typename M::V;
  // staging area: the earlier chunks' diagonal-block inverses for the sweep
  // (<= 14 blocks of 256), the panel rows 8 columns at a time ([row][8]), the
  // new diagonal block and the inversion scratch (2 x 1024)
  __shared__ T stage[14 * 256];
  __shared__ T xk[2][16 * CW];   // published X_k [row][col]
  __shared__ T crow_[2][4][CW];  // per wave: the row of its best pivot candidate
  __shared__ T cval[2][4];        // per wave: |candidate|
  __shared__ int ckey[2][4];      // per wave: candidate position (INT_MAX: none)
  __shared__ int pm[256];         // position -> original (leaf-local) row

  const int a = blockIdx.x;
  const int64_t o = leaf_off[a];
  const int m = (int)(leaf_off[a + 1] - o);
  const int tid0 = threadIdx.x, w0 = __builtin_amdgcn_readfirstlane(tid0 >> 6);
  T* F = lu + (inplace ? o : (int64_t)a * ldl * ldl);  // by original row while factoring (ld lul)
  T* IL = invl + (int64_t)a * 2 * (ldl / 16) * 256;
  int32_t* pv = piv + (int64_t)a * ldl;
  const int nbk = (m + 15) >> 4;
  const int nch = (m + CW - 1) / CW;

  for (int i = tid0; i < 256; i += kLuThreads) pm[i] = i;
  // zero padding outside m x m (never touched by the factorization)
  if (m < ldl && !inplace) {
    for (int j = 0; j < ldl; ++j)
      for (int i = tid0; i < ldl; i += kLuThreads)
        if (i >= m || j >= m) F[i + (int64_t)j * lul] = T(0);
  }
  __syncthreads();

  for (int c = 0; c < nch; ++c) {
    // lane coordinates are re-derived from opaque copies in every chunk so the
    // compiler cannot hoist lane-dependent addresses and constants out of the
    // chunk loop (they would otherwise stay live and spill)
    int tid = tid0, w = w0;
    asm volatile("" : "+v"(tid));
    asm volatile("" : "+s"(w));
    const int lane = tid & 63, li = lane & 15, lq = lane >> 4;
    const int c0 = CW * c;
    const int cw = min(CW, m - c0);
    // 1. load the chunk in the current row order
    V acc[4][CW / 16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int cb = 0; cb < CW / 16; ++cb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int row = 16 * (4 * q + w) + M::crow(lq, t);
          const int col = 16 * cb + li;
          acc[q][cb][t] = (row < m && col < cw) ? (T)D[o + pm[row] + (int64_t)(c0 + col) * ldd] : T(0);
        }
    // 2. sweep with the L blocks of the earlier chunks; their diagonal-block
    // inverses are staged in LDS first (the panel buffer is free until the
    // panel), so the owner's step waits on no global load
    const int nk = (CW / 16) * c;
    T* ILs = stage;
    for (int e = tid; e < nk * 256; e += kLuThreads) ILs[e] = IL[e];
    __syncthreads();
    for (int k = 0; k < nk; ++k) {
      T* xb = xk[k & 1];
      if ((k & 3) == w) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (4 * q + w == k) {
#pragma unroll
            for (int cb = 0; cb < CW / 16; ++cb) {
              T lv[4], bv[4];
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                lv[t] = ILs[k * 256 + li * 16 + M::crow(lq, t)];
                bv[t] = acc[q][cb][t];
              }
              const V nv = Mma16<T, BF>::mma(lv, bv, vzero<V>());
              acc[q][cb] = nv;
#pragma unroll
              for (int t = 0; t < 4; ++t) xb[M::crow(lq, t) * CW + 16 * cb + li] = nv[t];
            }
          }
      }
      // operands of this step's update are independent of X_k: load them
      // before the barrier (rows clamped in range, used only by active blocks)
      T av[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = min(4 * q + w, nbk - 1);
        const int prow = pm[16 * b + li];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) av[q][ks] = -F[prow + (int64_t)(16 * k + 4 * ks + lq) * lul];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = 4 * q + w;
        if (b > k && b < nbk) {  // uniform
          if constexpr (BF) {
#pragma unroll
            for (int cb = 0; cb < CW / 16; ++cb) {
              T xv[4];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) xv[ks] = xb[(4 * ks + lq) * CW + 16 * cb + li];
              acc[q][cb] = Mma16<T, true>::mma(av[q], xv, acc[q][cb]);
            }
          } else {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
#pragma unroll
              for (int cb = 0; cb < CW / 16; ++cb)
                acc[q][cb] = M::mma(av[q][ks], xb[(4 * ks + lq) * CW + 16 * cb + li], acc[q][cb]);
          }
        }
      }
    }
    // U rows above the panel are final
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int cb = 0; cb < CW / 16; ++cb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int row = 16 * (4 * q + w) + M::crow(lq, t);
          const int col = 16 * cb + li;
          if (row < m && row < c0 && col < cw) F[pm[row] + (int64_t)(c0 + col) * lul] = acc[q][cb][t];
        }
    // 3. panel factorization, one thread per panel row
    const int pr = m - c0;
    const bool own = tid < pr;
    int mypos = tid;
    bool done = false;
    const int orig = own ? pm[c0 + tid] : 0;
    // panel rows to the registers through LDS, 8 columns at a time
    T r[CW];
#pragma unroll
    for (int h = 0; h < CW / 8; ++h) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int row = 16 * (4 * q + w) + M::crow(lq, t);
          if (row < m && row >= c0 && (li >> 3) == (h & 1)) stage[(row - c0) * 8 + (li & 7)] = acc[q][h >> 1][t];
        }
      __syncthreads();
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) r[8 * h + cc] = own ? stage[tid * 8 + cc] : T(0);
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      if (j < cw) {
        // one barrier per column: each wave publishes its best candidate (value,
        // position, whole row); every thread then picks the winner of the four
        const int sb = j & 1;
        const bool cand = own && !done;
        T v = cand ? fabs(r[j]) : T(-1);
        if (cand && !(v == v)) v = T(INFINITY);  // a NaN can still be chosen
        T vmax;
        int key;
        wave_argmax(v, cand ? mypos : 0x7fffffff, vmax, key);
        v = vmax;
        if (cand && mypos == key) {
#pragma unroll
          for (int cc = 0; cc < CW; ++cc) crow_[sb][w][cc] = r[cc];
        }
        if (lane == 0) {
          cval[sb][w] = v;
          ckey[sb][w] = key;
        }
        __syncthreads();
        T bv = cval[sb][0];
        int bk = ckey[sb][0], bw = 0;
#pragma unroll
        for (int x = 1; x < 4; ++x)
          if (cval[sb][x] > bv || (cval[sb][x] == bv && ckey[sb][x] < bk)) {
            bv = cval[sb][x];
            bk = ckey[sb][x];
            bw = x;
          }
        const T* prow = crow_[sb][bw];
        if (cand) {
          if (mypos == bk) {  // this row is the pivot of column j
            done = true;
            pv[c0 + j] = c0 + bk;
            if (r[j] == T(0)) atomicMin(info, ((unsigned long long)a << 20) | (unsigned long long)(c0 + j));
            mypos = j;
          } else {
            if (mypos == j) mypos = bk;  // the row displaced by the interchange
            const T pivot = prow[j];
            if (pivot != T(0)) {
              const T l = r[j] * (T(1) / pivot);
              r[j] = l;
#pragma unroll
              for (int cc = j + 1; cc < CW; ++cc) r[cc] -= l * prow[cc];
            }
          }
        }
      }
    }
    // store the panel by original row and record the new row order; the rows
    // that became pivot rows also go to LDS as the chunk's 32 x 32 diagonal
    // block (pivoted order), from which the diagonal-block inverses are formed
    T* dblk = stage;  // [32][32] row-major; the panel no longer reads stage
    if (own) {
#pragma unroll
      for (int cc = 0; cc < CW; ++cc)
        if (cc < cw) F[orig + (int64_t)(c0 + cc) * lul] = r[cc];
      if (mypos < CW) {
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) dblk[mypos * CW + cc] = r[cc];
      }
    }
    __syncthreads();
    if (own) pm[c0 + mypos] = orig;
    // inverses of the new 16 x 16 diagonal blocks: threads 0..31 invert the
    // unit-lower L blocks, 32..63 the upper U blocks (one column each); rows
    // beyond m act as identity
    if (tid < 64) {
      const int half = (tid >> 4) & 1;
      int cc = tid & 15;
      asm volatile("" : "+v"(cc));  // keeps the identity columns from being hoisted out of the chunk loop
      const int kb = (CW / 16) * c + half;
      const int g0 = 16 * kb;
      const T* Bk = dblk + (16 * half) * CW + 16 * half;  // element (i, j) at Bk[i * CW + j]
      T* xs = stage + CW * CW + tid * 16;                  // this thread's column, in LDS (rolled loops: few registers)
      if (half < CW / 16 && kb < nbk) {
        if (tid < 32) {
#pragma unroll 1
          for (int i = 0; i < 16; ++i) {
            T sacc = (i == cc) ? T(1) : T(0);
            for (int jj = 0; jj < i; ++jj) {
              const T bv = Bk[i * CW + jj];
              sacc -= ((g0 + i < m) ? bv : T(0)) * xs[jj];
            }
            xs[i] = (i >= cc) ? sacc : T(0);
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) IL[kb * 256 + i * 16 + cc] = xs[i];
        } else {
#pragma unroll 1
          for (int i = 15; i >= 0; --i) {
            T sacc = (i == cc) ? T(1) : T(0);
            for (int jj = i + 1; jj < 16; ++jj) {
              const T bv = Bk[i * CW + jj];
              sacc -= ((g0 + i < m && g0 + jj < m) ? bv : T(0)) * xs[jj];
            }
            const T dv = Bk[i * CW + i];
            const T d = (g0 + i < m) ? dv : T(1);
            xs[i] = (i <= cc) ? sacc / d : T(0);
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) IL[(ldl / 16 + kb) * 256 + i * 16 + cc] = xs[i];
        }
      }
    } else if (tid < 64 + CW && c0 + tid - 64 < ldl) {
      const int j = tid - 64;
      udinv[(int64_t)a * ldl + c0 + j] = (j < cw) ? T(1) / dblk[j * CW + j] : T(1);
    }
    __syncthreads();
  }
  const int tid = tid0;
  // pivoted order: F[i, :] <- F[perm[i], :], 32 columns at a time; nothing
  // to do when no row moved
  const bool moved = tid < m && pm[tid] != tid;
  if (__syncthreads_or(moved)) {
    const int src = tid < m ? pm[tid] : tid;
    for (int g = 0; g < nch; ++g) {
      T r[CW];
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) {
        const int col = min(CW * g + cc, m - 1);
        r[cc] = F[min(src, m - 1) + (int64_t)col * lul];
      }
      __syncthreads();
      if (moved) {
#pragma unroll
        for (int cc = 0; cc < CW; ++cc)
          if (CW * g + cc < m) F[tid + (int64_t)(CW * g + cc) * lul] = r[cc];
      }
      __syncthreads();
    }
  }
  int32_t* pmo = perm + (int64_t)a * ldl;
  for (int i = tid; i < ldl; i += kLuThreads) {
    pmo[i] = i < m ? pm[i] : i;
    if (i >= m) pv[i] = i;
    if (i >= nch * CW) udinv[(int64_t)a * ldl + i] = T(1);  // beyond the last chunk of a short leaf
  }
}

template <typename T, typename S>
hipError_t launch_leaf_lu(hipStream_t s, int nleaf, int ldl, const int64_t* d_leaf_off, const S* D, int64_t ldd,
                          T* lu, int64_t lul, int inplace, int32_t* piv, int32_t* perm, T* udinv, T* invl,
                          unsigned long long* info, int bf) {
  if (nleaf == 0) return hipSuccess;
  if (ldl % 16 || ldl > 256) return hipErrorInvalidValue;
  if (inplace ? lul < ldl : lul != ldl) return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 4) {
    if (bf) {
      hipLaunchKernelGGL((leaf_lu_kernel<T, S, kCW, true>), dim3(nleaf), dim3(kLuThreads), 0, s, ldl, d_leaf_off, D,
                         ldd, lu, lul, inplace, piv, perm, udinv, invl, info);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((leaf_lu_kernel<T, S, kCW, false>), dim3(nleaf), dim3(kLuThreads), 0, s, ldl, d_leaf_off, D, ldd,
                     lu, lul, inplace, piv, perm, udinv, invl, info);
  return hipGetLastError();
}

template hipError_t launch_leaf_lu<double, double>(hipStream_t, int, int, const int64_t*, const double*, int64_t,
                                                   double*, int64_t, int, int32_t*, int32_t*, double*, double*,
                                                   unsigned long long*, int);
template hipError_t launch_leaf_lu<float, double>(hipStream_t, int, int, const int64_t*, const double*, int64_t,
                                                  float*, int64_t, int, int32_t*, int32_t*, float*, float*,
                                                  unsigned long long*, int);
template hipError_t launch_leaf_lu<float, float>(hipStream_t, int, int, const int64_t*, const float*, int64_t,
                                                 float*, int64_t, int, int32_t*, int32_t*, float*, float*,
                                                 unsigned long long*, int);

}  // namespace hodlr
