// FP64 HODLR matrix products, gradient assembly and refinement helpers.
//
// Matrix product (eq. "e:rank"): y_a = D_a x_a + sum_l U_a (V_b^T x_b) over
// the level-l ancestor-or-self a of each leaf and its sibling b.  The V^T x
// projections come from the level-pass product (per leaf tile, all R columns
// at once) followed by a pairwise tree sum; the apply kernel then forms
// [D_a | U(I_a, :)] [x_a ; G_a] on MFMA, G_a gathering each level's sibling
// projection.  A^T swaps U and V and transposes the leaf blocks.
//
// Gradients (dL/dA = -Lambda X^T restricted to D, U, V):
//   dD_a = -Lambda_a X_a^T,  dU(I_a, level l) = -Lambda_a (V_b^T X_b)^T,
//   dV(I_b, level l) = -X_b (U_a^T Lambda_a)^T.
#include "internal.h"

namespace hodlr {

constexpr int kMvThreads = 256;

__device__ __forceinline__ d4 mma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int crow64(int lq, int t) { return 4 * t + lq; }

// pairwise tree sum: out[i] = in[2i] + in[2i+1], blocks of `elems`
__global__ void tree_sum_kernel(int nnodes, int64_t elems, const double* __restrict__ in, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (e >= elems || i >= nnodes) return;
  out[(int64_t)i * elems + e] = in[(int64_t)(2 * i) * elems + e] + in[(int64_t)(2 * i + 1) * elems + e];
}

hipError_t launch_tree_sum(hipStream_t s, int nnodes, int64_t elems, const double* in, double* out) {
  if (nnodes == 0 || elems == 0) return hipSuccess;
  dim3 grid((unsigned)((elems + 255) / 256), (unsigned)nnodes);
  hipLaunchKernelGGL(tree_sum_kernel, grid, dim3(256), 0, s, nnodes, elems, in, out);
  return hipGetLastError();
}

// y(leaf rows, chunk) = op(D_a) x_a + U(I_a, :) G_a     (op = identity or transpose)
template <typename S, int TRANS, int NCB, bool FULL>
__global__ __launch_bounds__(kMvThreads) void matvec_apply_kernel(
    const int64_t* __restrict__ leaf_off, int L, const int32_t* __restrict__ rpre, int R, const S* __restrict__ D,
    int64_t ldd, const S* __restrict__ Ua, int64_t lda, const double* __restrict__ X, int64_t ldx,
    const double* __restrict__ tree, double* __restrict__ Y, int64_t ldy, int nrhs, int zchunks) {
  const int leaf = blockIdx.x / zchunks;
  const int zc = blockIdx.x % zchunks;
  const int64_t o = leaf_off[leaf];
  const int m = (int)(leaf_off[leaf + 1] - o);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lq = lane >> 4;
  const int c0 = zc * 64;
  const int wr0 = 64 * w;
  d4 acc[4][NCB];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = d4{0, 0, 0, 0};
  // One K-step of 4 columns: A operand rows of the leaf (clamped into range
  // and masked unless FULL), B operand from x or the level's projections.
  // Four steps' loads are issued before their MFMAs so several are in flight.
  auto kstep = [&](bool tr, const S* Am, int64_t ldA, int kcol, int kend, const double* Bm, int64_t ldB, int kofs,
                   double (&av)[4], double (&bv)[NCB]) {
    const int kk = kcol + lq, kc = FULL ? kk : min(kk, kend - 1);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int row = wr0 + 16 * rb + li, rc = FULL ? row : min(row, m - 1);
      const double v = tr ? (double)Am[o + kc + (int64_t)rc * ldA] : (double)Am[o + rc + (int64_t)kc * ldA];
      av[rb] = (FULL || (row < m && kk < kend)) ? v : 0.0;
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int col = c0 + 16 * cb + li;
      const double v = Bm[kofs + kc + (int64_t)min(col, nrhs - 1) * ldB];
      bv[cb] = ((FULL || kk < kend) && col < nrhs) ? v : 0.0;
    }
  };
  auto run = [&](bool tr, const S* Am, int64_t ldA, int kbeg, int kend, const double* Bm, int64_t ldB, int kofs) {
    int k0 = kbeg;
    for (; k0 + 16 <= kend; k0 += 16) {
      double av[4][4], bv[4][NCB];
#pragma unroll
      for (int u = 0; u < 4; ++u) kstep(tr, Am, ldA, k0 + 4 * u, kend, Bm, ldB, kofs, av[u], bv[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = mma64(av[u][rb], bv[u][cb], acc[rb][cb]);
    }
    for (; k0 < kend; k0 += 4) {
      double av[4], bv[NCB];
      kstep(tr, Am, ldA, k0, kend, Bm, ldB, kofs, av, bv);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = mma64(av[rb], bv[cb], acc[rb][cb]);
    }
  };
  // leaf block: rows of x are the leaf's rows
  run(TRANS, D, ldd, 0, m, X + o, ldx, 0);
  // low-rank blocks of every level: the sibling's projections V^T x
  for (int l = 1; l <= L; ++l) {
    const int cl0 = rpre[l - 1], cl1 = rpre[l];
    if (cl1 == cl0) continue;
    const int node = leaf >> (L - l);
    run(false, Ua, lda, cl0, cl1, tree + tree_slot(l, node ^ 1) * R * nrhs, R, 0);
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = wr0 + 16 * rb + crow64(lq, t);
        const int col = c0 + 16 * cb + li;
        if (row < m && col < nrhs) Y[o + row + (int64_t)col * ldy] = acc[rb][cb][t];
      }
}

template <typename S>
hipError_t launch_matvec_apply(hipStream_t s, int trans, int nleaf, int L, const int64_t* d_leaf_off,
                               const int32_t* d_rpre, int R, const S* D, int64_t ldd, const S* Ua, int64_t lda,
                               const double* X, int64_t ldx, const double* tree, double* Y, int64_t ldy, int nrhs,
                               int full) {
  if (nleaf == 0 || nrhs == 0) return hipSuccess;
  const int zchunks = (nrhs + 63) / 64;
  dim3 grid((unsigned)(nleaf * zchunks));
#define HODLR_MV(TR, NC)                                                                                        \
  if (full)                                                                                                       \
    hipLaunchKernelGGL((matvec_apply_kernel<S, TR, NC, true>), grid, dim3(kMvThreads), 0, s, d_leaf_off, L, d_rpre, \
                       R, D, ldd, Ua, lda, X, ldx, tree, Y, ldy, nrhs, zchunks);                                   \
  else                                                                                                            \
    hipLaunchKernelGGL((matvec_apply_kernel<S, TR, NC, false>), grid, dim3(kMvThreads), 0, s, d_leaf_off, L, d_rpre, \
                       R, D, ldd, Ua, lda, X, ldx, tree, Y, ldy, nrhs, zchunks)
  // chunks of 64 columns; up to 16 or 32 columns a narrower instance (one chunk, no padded MFMA columns)
  if (trans) {
    if (nrhs <= 16) { HODLR_MV(1, 1); } else if (nrhs <= 32) { HODLR_MV(1, 2); } else { HODLR_MV(1, 4); }
  } else {
    if (nrhs <= 16) { HODLR_MV(0, 1); } else if (nrhs <= 32) { HODLR_MV(0, 2); } else { HODLR_MV(0, 4); }
  }
#undef HODLR_MV
  return hipGetLastError();
}
template hipError_t launch_matvec_apply<double>(hipStream_t, int, int, int, const int64_t*, const int32_t*, int,
                                                const double*, int64_t, const double*, int64_t, const double*,
                                                int64_t, const double*, double*, int64_t, int, int);
template hipError_t launch_matvec_apply<float>(hipStream_t, int, int, int, const int64_t*, const int32_t*, int,
                                               const float*, int64_t, const float*, int64_t, const double*, int64_t,
                                               const double*, double*, int64_t, int, int);

// ---------------------------------------------------------------------------
// gradients
// ---------------------------------------------------------------------------
// dD_a(i, j) = add(o+i, j) - sum_k Lam(o+i, k) X(o+j, k) (add: FP64, ld ldadd, or null = 0);
// WG = (leaf, 64-column chunk of the block)
template <typename S>
__global__ __launch_bounds__(kMvThreads) void grad_leaf_kernel(const int64_t* __restrict__ leaf_off, int nchunks,
                                                               int nrhs, const double* __restrict__ X, int64_t ldx,
                                                               const double* __restrict__ Lam, int64_t ldl,
                                                               S* __restrict__ dD, int64_t ldd,
                                                               const double* __restrict__ add, int64_t ldadd) {
  const int leaf = blockIdx.x / nchunks, ch = blockIdx.x % nchunks;
  const int64_t o = leaf_off[leaf];
  const int m = (int)(leaf_off[leaf + 1] - o);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lq = lane >> 4;
  const int c0 = ch * 64;
  if (c0 >= m) return;
  const int wr0 = 64 * w;
  d4 acc[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = d4{0, 0, 0, 0};
  for (int k0 = 0; k0 < nrhs; k0 += 4) {
    const int kk = k0 + lq;
    double av[4], bv[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int row = wr0 + 16 * rb + li;
      av[rb] = (row < m && kk < nrhs) ? -Lam[o + row + (int64_t)kk * ldl] : 0.0;
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = c0 + 16 * cb + li;
      bv[cb] = (col < m && kk < nrhs) ? X[o + col + (int64_t)kk * ldx] : 0.0;
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = mma64(av[rb], bv[cb], acc[rb][cb]);
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = wr0 + 16 * rb + crow64(lq, t);
        const int col = c0 + 16 * cb + li;
        if (row < m && col < m)
          dD[o + row + (int64_t)col * ldd] = (S)((add ? add[o + row + (int64_t)col * ldadd] : 0.0) + acc[rb][cb][t]);
      }
}

template <typename S>
hipError_t launch_grad_leaf(hipStream_t s, int nleaf, int m_max, const int64_t* d_leaf_off, int nrhs,
                            const double* X, int64_t ldx, const double* Lam, int64_t ldl, S* dD, int64_t ldd,
                            const double* add, int64_t ldadd) {
  if (nleaf == 0) return hipSuccess;
  const int nchunks = (m_max + 63) / 64;
  hipLaunchKernelGGL(grad_leaf_kernel<S>, dim3((unsigned)(nleaf * nchunks)), dim3(kMvThreads), 0, s, d_leaf_off,
                     nchunks, nrhs, X, ldx, Lam, ldl, dD, ldd, add, ldadd);
  return hipGetLastError();
}
template hipError_t launch_grad_leaf<double>(hipStream_t, int, int, const int64_t*, int, const double*, int64_t,
                                             const double*, int64_t, double*, int64_t, const double*, int64_t);
template hipError_t launch_grad_leaf<float>(hipStream_t, int, int, const int64_t*, int, const double*, int64_t,
                                            const double*, int64_t, float*, int64_t, const double*, int64_t);

// out(I_leaf, c) = add(I_leaf, c) - sum_j Left(I_leaf, j) * S_l(c)[sib](c, j) for every column c of
// U_big / V_big (add: FP64 N x R with ld ldadd, or null = 0); the sum runs over j < nrhs, or with
// tri = 1 over the columns of the levels above c's level only (j < R_{l-1})
template <typename S>
__global__ __launch_bounds__(kMvThreads) void grad_gen_kernel(const int64_t* __restrict__ leaf_off, int L,
                                                              const int32_t* __restrict__ rpre, int R, int nchunks,
                                                              int nrhs, const double* __restrict__ Left, int64_t ldl,
                                                              const double* __restrict__ tree,
                                                              S* __restrict__ out, int64_t ldo,
                                                              const double* __restrict__ add, int64_t ldadd,
                                                              int tri) {
  const int leaf = blockIdx.x / nchunks, ch = blockIdx.x % nchunks;
  const int64_t o = leaf_off[leaf];
  const int m = (int)(leaf_off[leaf + 1] - o);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lq = lane >> 4;
  const int c0 = ch * 64;
  const int wr0 = 64 * w;
  // per column block cb: level, sibling block base
  const double* sb[4];
  int cvalid[4], klim[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int c = c0 + 16 * cb + li;
    cvalid[cb] = c < R;
    int l = 1;
    while (l < L && c >= rpre[l]) ++l;
    const int node = leaf >> (L - l);
    sb[cb] = cvalid[cb] ? tree + tree_slot(l, node ^ 1) * R * nrhs + c : tree;
    klim[cb] = tri ? min(nrhs, (int)rpre[l - 1]) : nrhs;
  }
  d4 acc[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = d4{0, 0, 0, 0};
  for (int k0 = 0; k0 < nrhs; k0 += 4) {
    const int kk = k0 + lq;
    double av[4], bv[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int row = wr0 + 16 * rb + li;
      av[rb] = (row < m && kk < nrhs) ? -Left[o + row + (int64_t)kk * ldl] : 0.0;
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) bv[cb] = (cvalid[cb] && kk < klim[cb]) ? sb[cb][(int64_t)kk * R] : 0.0;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = mma64(av[rb], bv[cb], acc[rb][cb]);
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = wr0 + 16 * rb + crow64(lq, t);
        const int col = c0 + 16 * cb + li;
        if (row < m && col < R)
          out[o + row + (int64_t)col * ldo] = (S)((add ? add[o + row + (int64_t)col * ldadd] : 0.0) + acc[rb][cb][t]);
      }
}

template <typename S>
hipError_t launch_grad_gen(hipStream_t s, int nleaf, int L, const int64_t* d_leaf_off, const int32_t* d_rpre, int R,
                           int nrhs, const double* Left, int64_t ldl, const double* tree, S* out, int64_t ldo,
                           const double* add, int64_t ldadd, int tri) {
  if (nleaf == 0 || R == 0) return hipSuccess;
  const int nchunks = (R + 63) / 64;
  hipLaunchKernelGGL(grad_gen_kernel<S>, dim3((unsigned)(nleaf * nchunks)), dim3(kMvThreads), 0, s, d_leaf_off, L,
                     d_rpre, R, nchunks, nrhs, Left, ldl, tree, out, ldo, add, ldadd, tri);
  return hipGetLastError();
}
template hipError_t launch_grad_gen<double>(hipStream_t, int, int, const int64_t*, const int32_t*, int, int,
                                            const double*, int64_t, const double*, double*, int64_t, const double*,
                                            int64_t, int);
template hipError_t launch_grad_gen<float>(hipStream_t, int, int, const int64_t*, const int32_t*, int, int,
                                           const double*, int64_t, const double*, float*, int64_t, const double*,
                                           int64_t, int);

// ---------------------------------------------------------------------------
// refinement helpers (FP64)
// ---------------------------------------------------------------------------
constexpr int kNormBlocks = 256;

// per (block, column): partial sum of squares and max |.| over a strided row range
__global__ void colnorm_partial_kernel(int64_t n, const double* __restrict__ X, int64_t ldx, double* __restrict__ part) {
  __shared__ double s2[256], si[256];
  const int j = blockIdx.y;
  double a2 = 0.0, ai = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = X[i + (int64_t)j * ldx];
    a2 += v * v;
    ai = fmax(ai, fabs(v));
  }
  s2[threadIdx.x] = a2;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s2[threadIdx.x] += s2[threadIdx.x + off];
      si[threadIdx.x] = fmax(si[threadIdx.x], si[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)j * gridDim.x + blockIdx.x) * 2] = s2[0];
    part[((int64_t)j * gridDim.x + blockIdx.x) * 2 + 1] = si[0];
  }
}
__global__ void colnorm_final_kernel(int nblk, int nrhs, const double* __restrict__ part, double* __restrict__ out2,
                                     double* __restrict__ outinf) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double a2 = 0.0, ai = 0.0;
  for (int b = 0; b < nblk; ++b) {
    a2 += part[((int64_t)j * nblk + b) * 2];
    ai = fmax(ai, part[((int64_t)j * nblk + b) * 2 + 1]);
  }
  out2[j] = sqrt(a2);
  outinf[j] = ai;
}

hipError_t launch_colnorms(hipStream_t s, int64_t n, int nrhs, const double* X, int64_t ldx, double* part,
                           double* out2, double* outinf) {
  if (nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(colnorm_partial_kernel, dim3(kNormBlocks, nrhs), dim3(256), 0, s, n, X, ldx, part);
  hipLaunchKernelGGL(colnorm_final_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, s, kNormBlocks, nrhs, part, out2,
                     outinf);
  return hipGetLastError();
}

template <typename T>
__global__ void scale_down_kernel(int64_t n, const double* __restrict__ Rr, int64_t ldr,
                                  const double* __restrict__ sc, T* __restrict__ out, int64_t ldo) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = sc[j] > 0.0 ? sc[j] : 1.0;
  out[i + (int64_t)j * ldo] = (T)(Rr[i + (int64_t)j * ldr] / d);
}
template <typename T>
hipError_t launch_scale_down(hipStream_t s, int64_t n, int nrhs, const double* Rr, int64_t ldr, const double* sc,
                             T* out, int64_t ldo) {
  if (nrhs == 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_down_kernel<T>, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, n, Rr, ldr, sc,
                     out, ldo);
  return hipGetLastError();
}
template hipError_t launch_scale_down<double>(hipStream_t, int64_t, int, const double*, int64_t, const double*,
                                              double*, int64_t);
template hipError_t launch_scale_down<float>(hipStream_t, int64_t, int, const double*, int64_t, const double*, float*,
                                             int64_t);

template <typename T>
__global__ void axpy_up_kernel(int64_t n, const T* __restrict__ d, int64_t ldd, const double* __restrict__ sc,
                               double* __restrict__ X, int64_t ldx) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double f = sc[j] > 0.0 ? sc[j] : 1.0;
  X[i + (int64_t)j * ldx] += (double)d[i + (int64_t)j * ldd] * f;
}
template <typename T>
hipError_t launch_axpy_up(hipStream_t s, int64_t n, int nrhs, const T* d, int64_t ldd, const double* sc, double* X,
                          int64_t ldx) {
  if (nrhs == 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_up_kernel<T>, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, n, d, ldd, sc, X,
                     ldx);
  return hipGetLastError();
}
template hipError_t launch_axpy_up<double>(hipStream_t, int64_t, int, const double*, int64_t, const double*, double*,
                                           int64_t);
template hipError_t launch_axpy_up<float>(hipStream_t, int64_t, int, const float*, int64_t, const double*, double*,
                                          int64_t);

// AX <- B - AX
__global__ void residual_kernel(int64_t n, const double* __restrict__ B, int64_t ldb, double* __restrict__ AX,
                                int64_t ldax) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  AX[i + (int64_t)j * ldax] = B[i + (int64_t)j * ldb] - AX[i + (int64_t)j * ldax];
}
hipError_t launch_residual(hipStream_t s, int64_t n, int nrhs, const double* B, int64_t ldb, double* AX, int64_t ldax) {
  if (nrhs == 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(residual_kernel, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, n, B, ldb, AX, ldax);
  return hipGetLastError();
}

template <typename T, typename S>
__global__ void convert_kernel(int64_t rows, const S* __restrict__ in, int64_t ldi, int64_t gsi, T* __restrict__ out,
                               int64_t ldo) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  out[i + (int64_t)j * ldo] = (T)in[group_row(i, gsi) + (int64_t)j * ldi];
}
template <typename T, typename S>
hipError_t launch_convert(hipStream_t s, int64_t rows, int cols, const S* in, int64_t ldi, T* out, int64_t ldo,
                          int64_t gsi) {
  if (rows == 0 || cols == 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<T, S>), dim3((unsigned)((rows + 255) / 256), cols), dim3(256), 0, s, rows, in, ldi,
                     gsi, out, ldo);
  return hipGetLastError();
}
template hipError_t launch_convert<double, double>(hipStream_t, int64_t, int, const double*, int64_t, double*, int64_t, int64_t);
template hipError_t launch_convert<double, float>(hipStream_t, int64_t, int, const float*, int64_t, double*, int64_t, int64_t);
template hipError_t launch_convert<float, double>(hipStream_t, int64_t, int, const double*, int64_t, float*, int64_t, int64_t);

}  // namespace hodlr
