// HODLR construction from a kernel function (Section II-B; the entries of
// Section I "Kernel matrices" and of the Laplace double layer, Section IV-B
// eq. "e:laplace_int"): exact leaf blocks, and every sibling block
// A(I_a, I_b) compressed by cross approximation with partial pivoting taken
// for r_l steps (the approximate partial-pivoted LU that the experiments of
// Section IV-A use):
//   for k = 1 .. r:
//     v = A(i_k, :) - sum_{l<k} u_l(i_k) v_l,   j_k = argmax |v|,  v_k = v / v(j_k)
//     u_k = A(:, j_k) - sum_{l<k} v_l(j_k) u_l,  i_{k+1} = argmax over unused rows |u_k|
// with i_1 = the block's first row, the lowest index on ties, and an
// exhausted step (v(j_k) = 0) giving u_k = v_k = 0.  U_a = [u_k] goes to rows
// I_a, V_b = [v_k] to rows I_b of the level's columns of U_big / V_big.
//
// All blocks of all levels advance together: step k is one launch for the
// residual rows (a workgroup per 1024-column tile of a block, writing v
// unnormalized and the tile's largest modulus) and one for the residual
// columns (each workgroup first reduces its block's row partials to j_k and
// the pivot value, normalizes its tile of v, then forms its tile of u and the
// tile's largest modulus over unused rows); the next row launch reduces those
// to i_{k+1}.  Partials are reduced in a fixed order (deterministic).
#include "internal.h"

#include <climits>

namespace hodlr {

namespace {

constexpr int kCsThreads = 256;
constexpr int kCsEpt = 4;
constexpr int kCsTile = kCsThreads * kCsEpt;  // elements of a block row / column per workgroup
constexpr double kPi = 3.141592653589793238462643383279502884;

__device__ __forceinline__ double kernel_offdiag(const ConstructKernel& k, int64_t p, int64_t q) {
  double d2 = 0.0, dx0 = 0.0, dx1 = 0.0;
  for (int d = 0; d < k.dim; ++d) {
    const double t = k.pts[p + d * k.ldp] - k.pts[q + d * k.ldp];
    d2 += t * t;
    if (d == 0) dx0 = t;
    if (d == 1) dx1 = t;
  }
  switch (k.kind) {
    case HODLR_KERNEL_GAUSS:
      return exp(-d2 / (2.0 * (k.ell * k.ell)));
    case HODLR_KERNEL_MATERN32: {
      const double s = sqrt(3.0) * sqrt(d2) / k.ell;
      return (1.0 + s) * exp(-s);
    }
    default: {  // Laplace double layer: w_q n_q . (x_p - x_q) / (2 pi |x_p - x_q|^2)
      const double num = k.nrm[q] * dx0 + k.nrm[q + k.ldp] * dx1;
      return num / (2.0 * kPi * d2) * k.w[q];
    }
  }
}

__device__ __forceinline__ double kernel_entry(const ConstructKernel& k, int64_t p, int64_t q) {
  if (p != q) return kernel_offdiag(k, p, q);
  const double d = k.kind == HODLR_KERNEL_LAPLACE_DL ? k.w[p] * k.kap[p] / (4.0 * kPi) : 1.0;
  return d + k.shift;
}

// (modulus, index) pairs: the larger modulus wins, the lower index on ties
__device__ __forceinline__ bool better(double a, int ia, double b, int ib) { return a > b || (a == b && ia < ib); }

// block-wide argmax of (a, idx, val) over kCsThreads threads; result in slot 0
__device__ __forceinline__ void block_argmax(double* sa, int* si, double* sv, int tid) {
  for (int s = kCsThreads / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (tid < s && better(sa[tid + s], si[tid + s], sa[tid], si[tid])) {
      sa[tid] = sa[tid + s];
      si[tid] = si[tid + s];
      if (sv) sv[tid] = sv[tid + s];
    }
  }
  __syncthreads();
}

}  // namespace

// leaf blocks: D(s0 + p, q) = A(s0 + p, s0 + q) for q < m, zero for m <= q < m_max
template <typename TS>
__global__ __launch_bounds__(kCsThreads) void construct_leaves_kernel(ConstructKernel k, const int64_t* __restrict__ off,
                                                                      int m_max, int ccols, TS* D, int64_t ldd) {
  const int a = blockIdx.x;
  const int64_t s0 = off[a];
  const int m = (int)(off[a + 1] - s0);
  const int p = threadIdx.x;
  if (p >= m) return;
  const int q0 = blockIdx.y * ccols;
  const int q1 = min(m_max, q0 + ccols);
  for (int q = q0; q < q1; ++q) D[(s0 + p) + (int64_t)q * ldd] = q < m ? (TS)kernel_entry(k, s0 + p, s0 + q) : TS(0);
}

// step k, residual rows: v(j) = A(i_k, j) - sum_{l<k} U(i_k, l) V(j, l) for the tile's columns
__global__ __launch_bounds__(kCsThreads) void aca_row_kernel(ConstructKernel kd, const AcaBlock* __restrict__ blocks,
                                                             const AcaTile* __restrict__ tiles, int k, int kmax,
                                                             const double* __restrict__ U, int64_t ldu, double* V,
                                                             int64_t ldv, const double* __restrict__ cp_abs,
                                                             const int* __restrict__ cp_idx, double* __restrict__ rp_abs,
                                                             double* __restrict__ rp_val, int* __restrict__ rp_idx,
                                                             int* __restrict__ piv) {
  const AcaTile tl = tiles[blockIdx.x];
  const AcaBlock b = blocks[tl.blk];
  if (k >= b.rank) return;
  __shared__ double sa[kCsThreads], sv[kCsThreads];
  __shared__ int si[kCsThreads];
  __shared__ double uk[HODLR_MAX_RANK];
  const int tid = threadIdx.x;
  int i = 0;
  if (k > 0) {  // i_k from the previous step's column partials of this block
    double best = -2.0;
    int bi = INT_MAX;
    for (int t = tid; t < b.ntile; t += kCsThreads)
      if (better(cp_abs[b.tile0 + t], cp_idx[b.tile0 + t], best, bi)) {
        best = cp_abs[b.tile0 + t];
        bi = cp_idx[b.tile0 + t];
      }
    sa[tid] = best;
    si[tid] = bi;
    block_argmax(sa, si, nullptr, tid);
    i = si[0];
  }
  if (tl.t == 0 && tid == 0) piv[(int64_t)tl.blk * kmax + k] = i;
  if (tid < k) uk[tid] = U[(b.r0 + i) + (int64_t)(b.col + tid) * ldu];
  __syncthreads();
  double best = -1.0, bval = 0.0;
  int bj = INT_MAX;
  const int64_t p = b.r0 + i;
  // the thread's kCsEpt columns advance together through l (independent
  // loads in flight); each column's terms are still subtracted in order of l
  double v[kCsEpt];
  const double* Vb = V + b.c0 + (int64_t)b.col * ldv;
  const int j0 = tl.t * kCsTile + tid;
  if (j0 + (kCsEpt - 1) * kCsThreads < b.n) {  // full tile (uniform)
#pragma unroll
    for (int e = 0; e < kCsEpt; ++e) v[e] = kernel_offdiag(kd, p, b.c0 + j0 + e * kCsThreads);
    for (int l = 0; l < k; ++l) {
      const double c = uk[l];
      const double* Vl = Vb + (int64_t)l * ldv + j0;
#pragma unroll
      for (int e = 0; e < kCsEpt; ++e) v[e] -= c * Vl[e * kCsThreads];
    }
  } else {
#pragma unroll
    for (int e = 0; e < kCsEpt; ++e) {
      const int j = j0 + e * kCsThreads;
      v[e] = 0.0;
      if (j < b.n) {
        v[e] = kernel_offdiag(kd, p, b.c0 + j);
        for (int l = 0; l < k; ++l) v[e] -= uk[l] * Vb[j + (int64_t)l * ldv];
      }
    }
  }
#pragma unroll
  for (int e = 0; e < kCsEpt; ++e) {
    const int j = j0 + e * kCsThreads;
    if (j < b.n) {
      V[(b.c0 + j) + (int64_t)(b.col + k) * ldv] = v[e];
      const double av = fabs(v[e]);
      if (av > best) {  // j increases along e: the first of equal moduli stays
        best = av;
        bj = j;
        bval = v[e];
      }
    }
  }
  sa[tid] = best;
  si[tid] = bj;
  sv[tid] = bval;
  block_argmax(sa, si, sv, tid);
  if (tid == 0) {
    rp_abs[tl.gtile] = sa[0];
    rp_idx[tl.gtile] = si[0];
    rp_val[tl.gtile] = sv[0];
  }
}

// step k, residual columns: j_k and the pivot value from the row partials,
// v_k = v / v(j_k) on the tile's columns, u(i) = A(i, j_k) - sum_{l<k} V(j_k, l) U(i, l)
// on the tile's rows, and the tile's largest |u| over rows not yet pivots
__global__ __launch_bounds__(kCsThreads) void aca_col_kernel(ConstructKernel kd, const AcaBlock* __restrict__ blocks,
                                                             const AcaTile* __restrict__ tiles, int k, int kmax,
                                                             double* U, int64_t ldu, double* V, int64_t ldv,
                                                             const double* __restrict__ rp_abs,
                                                             const double* __restrict__ rp_val,
                                                             const int* __restrict__ rp_idx, double* __restrict__ cp_abs,
                                                             int* __restrict__ cp_idx, const int* __restrict__ piv) {
  const AcaTile tl = tiles[blockIdx.x];
  const AcaBlock b = blocks[tl.blk];
  if (k >= b.rank) return;
  __shared__ double sa[kCsThreads], sv[kCsThreads];
  __shared__ int si[kCsThreads];
  __shared__ double vk[HODLR_MAX_RANK];
  __shared__ unsigned char used[kCsTile];
  const int tid = threadIdx.x;
  {
    double best = -2.0, bval = 0.0;
    int bj = INT_MAX;
    for (int t = tid; t < b.ntile; t += kCsThreads)
      if (better(rp_abs[b.tile0 + t], rp_idx[b.tile0 + t], best, bj)) {
        best = rp_abs[b.tile0 + t];
        bj = rp_idx[b.tile0 + t];
        bval = rp_val[b.tile0 + t];
      }
    sa[tid] = best;
    si[tid] = bj;
    sv[tid] = bval;
    block_argmax(sa, si, sv, tid);
  }
  const int j = si[0];
  const double delta = sv[0];
  const bool exhausted = delta == 0.0;
  const int row0 = tl.t * kCsTile;
#pragma unroll
  for (int e = 0; e < kCsEpt; ++e) {
    const int jj = row0 + e * kCsThreads + tid;
    if (jj < b.n) {
      double* pv = V + (b.c0 + jj) + (int64_t)(b.col + k) * ldv;
      *pv = exhausted ? 0.0 : *pv / delta;
    }
  }
  if (tid < k && !exhausted) vk[tid] = V[(b.c0 + j) + (int64_t)(b.col + tid) * ldv];
  for (int x = tid; x < kCsTile; x += kCsThreads) used[x] = 0;
  __syncthreads();
  if (tid <= k) {
    const int rel = piv[(int64_t)tl.blk * kmax + tid] - row0;
    if (rel >= 0 && rel < kCsTile) used[rel] = 1;
  }
  __syncthreads();
  double best = -2.0;
  int bi = INT_MAX;
  double u[kCsEpt];
  const double* Ub = U + b.r0 + (int64_t)b.col * ldu;
  const int i0 = row0 + tid;
  if (exhausted) {
#pragma unroll
    for (int e = 0; e < kCsEpt; ++e) u[e] = 0.0;
  } else if (i0 + (kCsEpt - 1) * kCsThreads < b.m) {  // full tile (uniform)
#pragma unroll
    for (int e = 0; e < kCsEpt; ++e) u[e] = kernel_offdiag(kd, b.r0 + i0 + e * kCsThreads, b.c0 + j);
    for (int l = 0; l < k; ++l) {
      const double c = vk[l];
      const double* Ul = Ub + (int64_t)l * ldu + i0;
#pragma unroll
      for (int e = 0; e < kCsEpt; ++e) u[e] -= c * Ul[e * kCsThreads];
    }
  } else {
#pragma unroll
    for (int e = 0; e < kCsEpt; ++e) {
      const int ii = i0 + e * kCsThreads;
      u[e] = 0.0;
      if (ii < b.m) {
        u[e] = kernel_offdiag(kd, b.r0 + ii, b.c0 + j);
        for (int l = 0; l < k; ++l) u[e] -= vk[l] * Ub[ii + (int64_t)l * ldu];
      }
    }
  }
#pragma unroll
  for (int e = 0; e < kCsEpt; ++e) {
    const int ii = row0 + e * kCsThreads + tid;
    if (ii < b.m) {
      U[(b.r0 + ii) + (int64_t)(b.col + k) * ldu] = u[e];
      const double sc = used[ii - row0] ? -1.0 : fabs(u[e]);
      if (sc > best) {
        best = sc;
        bi = ii;
      }
    }
  }
  sa[tid] = best;
  si[tid] = bi;
  block_argmax(sa, si, nullptr, tid);
  if (tid == 0) {
    cp_abs[tl.gtile] = sa[0];
    cp_idx[tl.gtile] = si[0];
  }
}

// FP64 n x c (ld lds) to the storage type (ld ldd)
template <typename TS>
__global__ __launch_bounds__(kCsThreads) void store_cols_kernel(int64_t n, const double* __restrict__ src, int64_t lds,
                                                                TS* dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * kCsThreads + threadIdx.x;
  if (i < n) dst[i + (int64_t)blockIdx.y * ldd] = (TS)src[i + (int64_t)blockIdx.y * lds];
}

template <typename TS>
hipError_t launch_construct_leaves(hipStream_t s, const ConstructKernel& k, int nleaf, const int64_t* d_off, int m_max,
                                   TS* D, int64_t ldd) {
  if (nleaf == 0 || m_max > kCsThreads) return hipErrorInvalidValue;
  constexpr int ccols = 16;
  hipLaunchKernelGGL(construct_leaves_kernel<TS>, dim3(nleaf, (m_max + ccols - 1) / ccols), dim3(kCsThreads), 0, s, k,
                     d_off, m_max, ccols, D, ldd);
  return hipGetLastError();
}
template hipError_t launch_construct_leaves<double>(hipStream_t, const ConstructKernel&, int, const int64_t*, int,
                                                    double*, int64_t);
template hipError_t launch_construct_leaves<float>(hipStream_t, const ConstructKernel&, int, const int64_t*, int,
                                                   float*, int64_t);

int aca_tile_elems() { return kCsTile; }

hipError_t launch_aca_step(hipStream_t s, const ConstructKernel& k, int ntiles, const AcaBlock* blocks,
                           const AcaTile* tiles, int step, int kmax, double* U, int64_t ldu, double* V, int64_t ldv,
                           AcaPartials p) {
  if (ntiles == 0) return hipSuccess;
  if (kmax > HODLR_MAX_RANK) return hipErrorInvalidValue;
  hipLaunchKernelGGL(aca_row_kernel, dim3(ntiles), dim3(kCsThreads), 0, s, k, blocks, tiles, step, kmax,
                     (const double*)U, ldu, V, ldv, (const double*)p.cp_abs, (const int*)p.cp_idx, p.rp_abs, p.rp_val,
                     p.rp_idx, p.piv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(aca_col_kernel, dim3(ntiles), dim3(kCsThreads), 0, s, k, blocks, tiles, step, kmax, U, ldu, V,
                     ldv, (const double*)p.rp_abs, (const double*)p.rp_val, (const int*)p.rp_idx, p.cp_abs, p.cp_idx,
                     (const int*)p.piv);
  return hipGetLastError();
}

template <typename TS>
hipError_t launch_store_cols(hipStream_t s, int64_t n, int ncols, const double* src, int64_t lds, TS* dst,
                             int64_t ldd) {
  if (n == 0 || ncols == 0) return hipSuccess;
  hipLaunchKernelGGL(store_cols_kernel<TS>, dim3((unsigned)((n + kCsThreads - 1) / kCsThreads), ncols),
                     dim3(kCsThreads), 0, s, n, src, lds, dst, ldd);
  return hipGetLastError();
}
template hipError_t launch_store_cols<float>(hipStream_t, int64_t, int, const double*, int64_t, float*, int64_t);

}  // namespace hodlr
