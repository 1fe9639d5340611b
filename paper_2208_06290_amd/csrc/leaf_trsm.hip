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
// One workgroup per (block, chunk of columns).  The chunk (<= 256 rows)
// stays in MFMA accumulators for the whole solve: wave w of NW owns the
// 16-row blocks b with b % NW == w.  The inverses of the 16 x 16 diagonal
// blocks of L and U come with the factorization, so every block step is a
// contraction: the owning wave forms X_k = inv(M_kk) B_k, publishes X_k
// through LDS (double buffered, one barrier per step), and every wave applies
// B_b -= M_bk X_k to its blocks on MFMA; the factor operands and the next
// owner's inverted diagonal block are fetched before the barrier.  The
// products run transposed (X^T = B^T M^{-T}) so that accumulator rows are
// matrix rows on the lanes: every global load and store covers whole
// 128-byte lines.  Leaf blocks take 32-column chunks with 128 registers per
// lane (four workgroups per CU: the steps are short and latency-bound, so
// more resident workgroups pay more than wider chunks).
#include "mfma.h"

namespace hodlr {

constexpr int kTwLd = 17;  // padded row length of the owner's 16 x 16 turn-around buffer

// Resident workgroups per CU: four waves with accumulators of at most 64
// registers per lane (4 blocks x 2 column blocks of FP64, or 4 x 4 of FP32)
// keep four workgroups per CU, wider chunks two; eight waves two, or one.
template <typename T, int NW, int NQ, int NCB>
constexpr int trsm_occupancy() {
  return NW == 4 ? (NQ * NCB * (int)sizeof(T) <= 64 ? 4 : 2) : (NCB <= 2 ? 2 : 1);
}

template <typename T, typename S, int TRANS, int NW, int NQ, int NCB, bool BF>
__global__ __launch_bounds__(64 * NW, (trsm_occupancy<T, NW, NQ, NCB>())) void trsm_kernel(int ldl, const int64_t* __restrict__ leaf_off,
                                                             int64_t ostride, int mfix, const T* lu, int64_t lul,
                                                             int inplace, const int32_t* __restrict__ perm,
                                                             const T* __restrict__ dinv, const S* B, int64_t ldb,
                                                             T* X, int64_t ldx, int ncols, int nchunks, int64_t gsb,
                                                             int64_t gsx) {
  using M = Mfma<T>;
  using V = typename M::V;
  constexpr int kThreads = 64 * NW;
  constexpr int kBlocks = NW * NQ;  // 16-row blocks of a block (row block b is owned by wave b % NW)
  constexpr int kCwT = 16 * NCB;     // columns of a chunk
  __shared__ T xk[2][16 * kCwT];   // published block X_k: [row][col]
  __shared__ T tw[NW][16 * kTwLd];  // per-wave turn-around of the owner's block

  const int lid = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int a = lid / nchunks;
  const int chunk = lid % nchunks;
  int64_t o;
  int m;
  if (leaf_off) {
    o = leaf_off[a];
    m = (int)(leaf_off[a + 1] - o);
  } else {
    o = (int64_t)a * ostride;
    m = mfix;
  }
  // first row of the block in B and X (row i of an operand at (i >> 8) gs + (i & 255); a block
  // never crosses a 256-row boundary of an operand in the row-group blocked layout)
  const S* Bb = B + group_row(o, gsb);
  T* Xb = X + group_row(o, gsx);
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lq = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c0 = chunk * kCwT;
  const int nbk = (m + 15) >> 4;
  const T* F = lu + (inplace ? o : (int64_t)a * ldl * ldl);  // ld lul
  const int32_t* pm = perm + (int64_t)a * ldl;
  const int nbd = ldl >> 4;
  const T* DI = dinv + (int64_t)a * 2 * nbd * 256;  // [0][kb]: inv(L_kk), [1][kb]: inv(U_kk)
  T* twv = tw[w];

  // B operand of X_k^T = B_k^T inv(M_kk)^T: inv(M_kk)(li, 4 ks + lq) for ks = 0..3,
  // read from the factorization's inverted diagonal blocks (sweep 0 is L
  // (trans 0) or U^T (trans 1), sweep 1 is U or L^T)
  auto load_inv = [&](int sweep, int k, T (&iv)[4]) {
    const int which = TRANS ? 1 - sweep : sweep;
    const T* src = DI + ((int64_t)which * nbd + k) * 256;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int j = 4 * ks + lq;
      iv[ks] = TRANS ? src[j * 16 + li] : src[li * 16 + j];
    }
  };

  // The chunk is held transposed: accumulator block (q, cb), register t holds
  // X(16 (NW q + w) + li, c0 + 16 cb + crow(lq, t)), so the 16 lanes of a row
  // group touch 16 consecutive rows of one column (whole 128-byte lines).
  V acc[NQ][NCB];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int row = 16 * (NW * q + w) + li;
    const int rowc = min(row, m - 1);
    const int src = TRANS ? rowc : pm[rowc];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = c0 + 16 * cb + M::crow(lq, t);
        const T v = (T)Bb[src + (int64_t)min(col, ncols - 1) * ldb];
        acc[q][cb][t] = (row < m && col < ncols) ? v : T(0);
      }
  }
  __syncthreads();  // B may alias X: all loads of the chunk precede any store

  // X_k^T = B_k^T inv(M_kk)^T for the wave owning block k (accumulator block
  // q): the block turns around through LDS to become the A operand; the
  // result stays in the accumulators and is published as X_k[row][col]
  auto owner = [&](int q, const T (&iv)[4], T* xb) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int t = 0; t < 4; ++t) twv[li * kTwLd + M::crow(lq, t)] = acc[q][cb][t];
      T tv[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) tv[ks] = twv[(4 * ks + lq) * kTwLd + li];
      const V nv = Mma16<T, BF>::mma(tv, iv, vzero<V>());
      acc[q][cb] = nv;
#pragma unroll
      for (int t = 0; t < 4; ++t) xb[li * kCwT + 16 * cb + M::crow(lq, t)] = nv[t];
    }
  };
  // B_b^T -= X_k^T M_bk^T on accumulator block q2
  auto update = [&](int q2, const T (&av)[NQ][4], const T* xb) {
    if constexpr (BF) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        T xv[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) xv[ks] = xb[(4 * ks + lq) * kCwT + 16 * cb + li];
        acc[q2][cb] = Mma16<T, true>::mma(xv, av[q2], acc[q2][cb]);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[q2][cb] = M::mma(xb[(4 * ks + lq) * kCwT + 16 * cb + li], av[q2][ks], acc[q2][cb]);
    }
  };

  // The steps are unrolled so that every block index is a compile-time
  // constant; steps past the last block of a short leaf are skipped (uniform).
#pragma clang loop unroll(full)
  for (int sweep = 0; sweep < 2; ++sweep) {

#pragma clang loop unroll(full)
    for (int st = 0; st < kBlocks; ++st) {
      const int k = sweep == 0 ? st : kBlocks - 1 - st;
      if (k < nbk) {  // uniform
        const int q = k / NW, wk = k % NW;
        // step index within the sweep decides the X buffer (sweep 1 starts at nbk - 1)
        const int sidx = sweep == 0 ? k : nbk - 1 - k;
        T* xb = xk[sidx & 1];
        T* xn = xk[(sidx + 1) & 1];
        // the first step's X_k is formed here, later ones one step ahead (look-ahead)
        if (sidx == 0 && w == wk) {
          T iv0[4];
          load_inv(sweep, k, iv0);
          owner(q, iv0, xb);
        }
        // the factor operands M(16 b + li, 16 k + 4 ks + lq) of this wave's blocks
        // on the far side of k do not depend on X_k: fetched before the barrier
        // (clamped in range, no branches)
        T av[NQ][4];
#pragma unroll
        for (int q2 = 0; q2 < NQ; ++q2) {
          if (sweep == 0 ? q2 < q : q2 > q) continue;  // never on the far side: compile time
          const int b = min(NW * q2 + w, nbk - 1);
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const int i = 16 * b + li, j = 16 * k + 4 * ks + lq;
            av[q2][ks] = -(TRANS ? F[j + (int64_t)i * lul] : F[i + (int64_t)j * lul]);
          }
        }
        // look-ahead: the wave owning the next block updates it first and forms
        // X_next at once, so the next step starts without waiting for it
        const int kn = sweep == 0 ? k + 1 : k - 1;
        const bool nxt = sweep == 0 ? kn < nbk : kn >= 0;
        const int qn = kn / NW, wn = kn % NW;
        const bool la = nxt && w == wn;  // uniform
        T ivn[4];
        if (la) load_inv(sweep, kn, ivn);  // fetched before the barrier too
        __syncthreads();
        if (la) {
          update(qn, av, xb);
          owner(qn, ivn, xn);
        }
#pragma unroll
        for (int q2 = 0; q2 < NQ; ++q2) {
          if (sweep == 0 ? q2 < q : q2 > q) continue;
          const int b = NW * q2 + w;
          const bool act = (sweep == 0 ? (q2 > q || w > wk) : (q2 < q || w < wk)) && b < nbk &&
                           !(la && q2 == qn);  // uniform
          if (act) update(q2, av, xb);
        }
      }
    }
  }

  // store (the adjoint scatters rows through the permutation)
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int row = 16 * (NW * q + w) + li;
    if (row < m) {
      const int dst = TRANS ? pm[row] : row;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int col = c0 + 16 * cb + M::crow(lq, t);
          if (col < ncols) Xb[dst + (int64_t)col * ldx] = acc[q][cb][t];
        }
    }
  }
}

template <typename T, typename S>
static hipError_t launch_trsm(hipStream_t s, int trans, int nblk, int ldl, const int64_t* d_off, int64_t ostride,
                              int mfix, const T* lu, int64_t lul, int inplace, const int32_t* perm, const T* dinv,
                              const S* B, int64_t ldb, T* X, int64_t ldx, int ncols, int64_t gsb, int64_t gsx,
                              int bf) {
  if (nblk == 0 || ncols == 0) return hipSuccess;
  if (ldl % 16 || ldl > 256) return hipErrorInvalidValue;
  if (inplace ? (lul < ldl || !d_off) : lul != ldl) return hipErrorInvalidValue;
  // blocks of at most 64 rows (coupling systems): one 16-row block per wave,
  // chunks of 128 columns for few blocks and of 64 (twice the workgroups per
  // CU) for many; otherwise four blocks per wave and 32 columns
  const int nq = ldl <= 64 ? 1 : 4;
  // 4-byte elements: 64-column chunks of the leaf blocks hold as many
  // accumulator registers as 32 FP64 columns (four workgroups per CU), with
  // half the chunks and half the re-reads of each leaf's factors
  const int wide = sizeof(T) == 4 && nq == 4 && ncols > 32 ? 64 : 32;
  const int cw = nq == 1 ? (ncols > 64 && nblk < 512 ? 128 : ncols > 16 ? 64 : 16) : (ncols > 16 ? wide : 16);
  const int nchunks = (ncols + cw - 1) / cw;
  const int64_t grid = (int64_t)nblk * nchunks;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
#define HODLR_TS_B(TR, NW, NQ, NC, BFV)                                                                             \
  hipLaunchKernelGGL((trsm_kernel<T, S, TR, NW, NQ, NC, BFV>), dim3((unsigned)grid), dim3(64 * NW), 0, s, ldl, d_off, \
                     ostride, mfix, lu, lul, inplace, perm, dinv, B, ldb, X, ldx, ncols, nchunks, gsb, gsx)
#define HODLR_TS(TR, NW, NQ, NC) HODLR_TS_B(TR, NW, NQ, NC, false)
  // the 64-column leaf instance exists for 4-byte elements only
#define HODLR_TS_64(TR)                                \
  do {                                                 \
    if constexpr (sizeof(T) == 4) HODLR_TS(TR, 4, 4, 4); \
  } while (0)
  // up to 64 rows: 4 waves, one block each; up to 256 rows: 4 waves with four
  // blocks each for wide right-hand sides, 8 waves with two each for narrow ones
#define HODLR_TS_W(TR)                         \
  if (nq == 1) {                               \
    if (cw == 128) HODLR_TS(TR, 4, 1, 8);      \
    else if (cw == 64) HODLR_TS(TR, 4, 1, 4);  \
    else HODLR_TS(TR, 4, 1, 1);                \
  } else {                                     \
    if (cw == 64) HODLR_TS_64(TR);             \
    else if (cw == 32) HODLR_TS(TR, 4, 4, 2);  \
    else HODLR_TS(TR, 8, 2, 1);                \
  }
  // bfloat16 operands (FP32 factors and accumulation): the leaf solve of a
  // BF16 factorization
  bool done = false;
  if constexpr (sizeof(T) == 4) {
    if (bf && !trans && nq == 4) {
      if (cw == 64) HODLR_TS_B(0, 4, 4, 4, true);
      else if (cw == 32) HODLR_TS_B(0, 4, 4, 2, true);
      else HODLR_TS_B(0, 8, 2, 1, true);
      done = true;
    }
  }
  if (done) {
  } else if (trans) {
    HODLR_TS_W(1)
  } else {
    HODLR_TS_W(0)
  }
#undef HODLR_TS_W
#undef HODLR_TS_64
#undef HODLR_TS
#undef HODLR_TS_B
  return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_leaf_trsm(hipStream_t s, int trans, int nleaf, int ldl, const int64_t* d_leaf_off, const T* lu,
                            int64_t lul, int inplace, const int32_t* perm, const T* dinv, const S* B, int64_t ldb,
                            T* X, int64_t ldx, int ncols, int64_t gsb, int64_t gsx, int bf) {
  return launch_trsm<T, S>(s, trans, nleaf, ldl, d_leaf_off, 0, 0, lu, lul, inplace, perm, dinv, B, ldb, X, ldx, ncols,
                           gsb, gsx, bf);
}

template <typename T>
hipError_t launch_block_trsm(hipStream_t s, int trans, int nblk, int ldl, int m, int64_t ostride, const T* lu,
                             const int32_t* perm, const T* dinv, T* X, int64_t ldx, int ncols) {
  return launch_trsm<T, T>(s, trans, nblk, ldl, nullptr, ostride, m, lu, ldl, 0, perm, dinv, X, ldx, X, ldx, ncols,
                           256, 256, 0);
}

template hipError_t launch_leaf_trsm<double, double>(hipStream_t, int, int, int, const int64_t*, const double*,
                                                     int64_t, int, const int32_t*, const double*, const double*,
                                                     int64_t, double*, int64_t, int, int64_t, int64_t, int);
template hipError_t launch_leaf_trsm<float, double>(hipStream_t, int, int, int, const int64_t*, const float*,
                                                    int64_t, int, const int32_t*, const float*, const double*,
                                                    int64_t, float*, int64_t, int, int64_t, int64_t, int);
template hipError_t launch_leaf_trsm<float, float>(hipStream_t, int, int, int, const int64_t*, const float*,
                                                   int64_t, int, const int32_t*, const float*, const float*,
                                                   int64_t, float*, int64_t, int, int64_t, int64_t, int);
template hipError_t launch_block_trsm<double>(hipStream_t, int, int, int, int, int64_t, const double*,
                                              const int32_t*, const double*, double*, int64_t, int);
template hipError_t launch_block_trsm<float>(hipStream_t, int, int, int, int, int64_t, const float*, const int32_t*,
                                             const float*, float*, int64_t, int);

}  // namespace hodlr
