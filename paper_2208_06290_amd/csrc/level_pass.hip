// Fused per-level pass over row tiles (Alg. "a:gpuf" lines with batched_gemm,
// Alg. "a:gpus" lines with batched_gemm, restated on row tiles):
//
//   update : Z(tile, 0:nz) -= A1(tile, 0:ka) * W_node(0:ka, 0:nz)
//            factor: Y_big(I_a, 1:R_l) -= Y_a W_a        (eq. "e:node2")
//            solve : x(I_a) -= Y_a w_a                    (eq. "e:node4")
//   product: P_tile(0:kb, 0:nz) = B1(tile, 0:kb)^T * Z(tile, 0:nz)
//            the partial sums of V^T Y (eq. "e:node1" right side and the T
//            blocks of eq. "e:k") or of V^T x (eq. "e:node3") for the next level
//
// Both run on MFMA (f64 16x16x4 or f32 16x16x4).  The updated Z tile stays in
// the accumulator registers and feeds the product directly as B operand: in
// the accumulator layout each 4-register group holds 4 rows x 16 columns,
// exactly one K-step of the product.
//
// Workgroup = 256 threads = 4 waves; tile <= 256 rows (wave w owns rows
// 64w..64w+63), one chunk of 64 columns of Z and one chunk of <= 64 columns
// of B1; the four waves' partial products are summed in LDS in fixed order.
#include "mfma.h"

namespace hodlr {

constexpr int kLpThreads = 256;

template <typename TZ, typename SA, typename SB, int MB>
__global__ __launch_bounds__(kLpThreads, 2) void level_pass_kernel(const Tile* __restrict__ tiles, int zchunks,
                                                                   int bchunks, TZ* Z, int64_t ldz, int nz,
                                                                   const SA* __restrict__ A1, int64_t lda, int ka,
                                                                   const TZ* __restrict__ W, int64_t w_ld,
                                                                   int64_t w_pstride, int node_shift,
                                                                   const SB* __restrict__ B1, int64_t ldb,
                                                                   int kb_total, TZ* __restrict__ P) {
  using M = Mfma<TZ>;
  using V = typename M::V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TZ* Ws = reinterpret_cast<TZ*>(smem_raw);   // update phase: W chunk [k][64]
  TZ* red = reinterpret_cast<TZ*>(smem_raw);  // product phase: [4 waves][MB*16][64]

  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  const int bchunk = (int)(lid % bchunks);
  const int zchunk = (int)((lid / bchunks) % zchunks);
  const int64_t tile = lid / ((int64_t)bchunks * zchunks);
  const Tile tl = tiles[tile];
  const int64_t row0 = tl.row0;
  const int nrows = tl.nrows;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lq = lane >> 4;
  const int c0 = zchunk * 64;
  const int ncb = min(4, (nz - c0 + 15) >> 4);
  const int wr0 = 64 * w;  // first tile row of this wave
  const int nks = (ka + 3) >> 2;

  if (ka > 0) {
    const int nd = tl.node >> node_shift;
    const TZ* Wn = W + (int64_t)(nd >> 1) * w_pstride + (int64_t)(nd & 1) * ka;
    for (int e = tid; e < 64 * 4 * nks; e += kLpThreads) {  // rows padded to a whole K-step with zeros
      const int c = e % 64, k = e / 64;
      Ws[e] = (k < ka && c0 + c < nz) ? Wn[k + (int64_t)(c0 + c) * w_ld] : TZ(0);
    }
    __syncthreads();
  }

  auto load_z = [&](int rb, V (&dst)[4]) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = wr0 + 16 * rb + M::crow(lq, t);
        const int col = c0 + 16 * cb + li;
        dst[cb][t] = (cb < ncb && row < nrows && col < nz) ? Z[row0 + row + (int64_t)col * ldz] : TZ(0);
      }
  };

  const int kc0 = bchunk * 64;
  const int kb = kb_total > 0 ? min(64, kb_total - kc0) : 0;
  V pacc[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) pacc[mb][cb] = vzero<V>();

  V acc[4], nxt[4];
  load_z(0, nxt);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = nxt[cb];
    if (rb < 3) load_z(rb + 1, nxt);  // next row block in flight while this one computes
    if (ka > 0) {
      const int row = wr0 + 16 * rb + li;
      for (int ks = 0; ks < nks; ++ks) {
        const int kk = 4 * ks + lq;
        const TZ a = (row < nrows && kk < ka) ? -(TZ)A1[row0 + row + (int64_t)kk * lda] : TZ(0);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          if (cb < ncb) acc[cb] = M::mma(a, Ws[kk * 64 + 16 * cb + li], acc[cb]);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int rr = wr0 + 16 * rb + M::crow(lq, t);
          const int col = c0 + 16 * cb + li;
          if (cb < ncb && rr < nrows && col < nz) Z[row0 + rr + (int64_t)col * ldz] = acc[cb][t];
        }
    }
    if (kb > 0) {
      // the accumulator register t holds exactly the B operand (4 rows x 16 columns) of one K-step
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int rr = wr0 + 16 * rb + M::crow(lq, t);
        TZ bo[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int kr = 16 * mb + li;
          bo[mb] = (rr < nrows && kr < kb) ? (TZ)B1[row0 + rr + (int64_t)(kc0 + kr) * ldb] : TZ(0);
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            if (cb < ncb) pacc[mb][cb] = M::mma(bo[mb], acc[cb][t], pacc[mb][cb]);
      }
    }
  }

  if (kb > 0) {
    constexpr int kRows = MB * 16;
    if (ka > 0) __syncthreads();  // W chunk no longer read: its LDS becomes the reduction buffer
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int kr = 16 * mb + M::crow(lq, t);
          red[(w * kRows + kr) * 64 + 16 * cb + li] = pacc[mb][cb][t];
        }
    __syncthreads();
    TZ* Pt = P + tile * (int64_t)kb_total * nz;
    for (int e = tid; e < kb * 64; e += kLpThreads) {
      const int kr = e % kb, cw = e / kb;
      const int col = c0 + cw;
      if (col < nz) {
        TZ sum = red[(0 * kRows + kr) * 64 + cw];
        sum += red[(1 * kRows + kr) * 64 + cw];
        sum += red[(2 * kRows + kr) * 64 + cw];
        sum += red[(3 * kRows + kr) * 64 + cw];
        Pt[(kc0 + kr) + (int64_t)col * kb_total] = sum;
      }
    }
  }
}

template <typename TZ, typename SA, typename SB>
hipError_t launch_level_pass(hipStream_t s, int ntiles, const Tile* tiles, TZ* Z, int64_t ldz, int nz,
                             const SA* A1, int64_t lda, int ka, const TZ* W, int64_t w_ld, int64_t w_pstride,
                             int node_shift, const SB* B1, int64_t ldb, int kb, TZ* P) {
  if (ntiles == 0 || nz == 0 || (ka == 0 && kb == 0)) return hipSuccess;
  const int zchunks = (nz + 63) / 64;
  const int bchunks = kb > 0 ? (kb + 63) / 64 : 1;
  if (ka > 0 && bchunks > 1) return hipErrorInvalidValue;  // an update must run once per element
  const int64_t grid = (int64_t)ntiles * zchunks * bchunks;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  const int mbn = kb > 0 ? (min(kb, 64) + 15) / 16 : 1;
  const size_t smem_red = kb > 0 ? sizeof(TZ) * 4 * 16 * mbn * 64 : 0;
  const size_t smem_w = ka > 0 ? sizeof(TZ) * 64 * (size_t)((ka + 3) / 4 * 4) : 0;
  const size_t smem = smem_red > smem_w ? smem_red : smem_w;
#define HODLR_LP(MBV)                                                                                        \
  {                                                                                                          \
    auto k = level_pass_kernel<TZ, SA, SB, MBV>;                                                             \
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem); \
    if (e != hipSuccess) return e;                                                                           \
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kLpThreads), smem, s, tiles, zchunks, bchunks, Z, ldz, nz, \
                       A1, lda, ka, W, w_ld, w_pstride, node_shift, B1, ldb, kb, P);                                    \
  }
  switch (mbn) {
    case 1: HODLR_LP(1) break;
    case 2: HODLR_LP(2) break;
    case 3: HODLR_LP(3) break;
    default: HODLR_LP(4) break;
  }
#undef HODLR_LP
  return hipGetLastError();
}

#define HODLR_LP_INST(TZ, SA, SB)                                                                             \
  template hipError_t launch_level_pass<TZ, SA, SB>(hipStream_t, int, const Tile*, TZ*, int64_t, int, const SA*, \
                                                    int64_t, int, const TZ*, int64_t, int64_t, int,           \
                                                    const SB*, int64_t, int, TZ*);
HODLR_LP_INST(double, double, double)
HODLR_LP_INST(float, float, double)
HODLR_LP_INST(float, double, float)
HODLR_LP_INST(float, float, float)
HODLR_LP_INST(double, double, float)
#undef HODLR_LP_INST

}  // namespace hodlr
