// Sign and logarithm of |det A| from the stored factors (Section III-E,
// "Determinant"): with the product form A = D F_L ... F_1 of that section,
// det A = prod over leaves of det D_a times prod over parents of det F_g, and
// by Sylvester's determinant theorem det F_g = det [[I, T_b], [T_a, I]] with
// T = V^T Y, which is K_g = [[T_a, I], [I, T_b]] with its two r-row blocks
// exchanged: det F_g = (-1)^r det K_g.  Each LU with partial pivoting gives
// det = (-1)^(interchanges) prod of the pivots.
//
// Stage 1: one workgroup per item (leaf or parent) sums log|pivot| in FP64
// and counts negative pivots, interchanges and (for a parent) r, modulo 2.
// Stage 2: one workgroup adds the items in a fixed order, so the result is
// the same on every run.
#include <algorithm>

#include "internal.h"

namespace hodlr {

constexpr int kLdThreads = 256;

template <int NT>
__device__ __forceinline__ void block_sum(double& s, int& par, double* ls, int* lp) {
  const int tid = threadIdx.x;
  ls[tid] = s;
  lp[tid] = par;
  __syncthreads();
#pragma unroll
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      ls[tid] += ls[tid + h];
      lp[tid] ^= lp[tid + h];
    }
    __syncthreads();
  }
  s = ls[0];
  par = lp[0];
}

template <typename T>
__global__ __launch_bounds__(kLdThreads) void logdet_items_kernel(int nleaf, int ldl, const int64_t* __restrict__ leaf_off,
                                                                  const T* __restrict__ udinv,
                                                                  const int32_t* __restrict__ piv,
                                                                  const T* __restrict__ Kud,
                                                                  const int32_t* __restrict__ Kpiv, LogdetLevels lv,
                                                                  double* __restrict__ item_log,
                                                                  int* __restrict__ item_par) {
  __shared__ double ls[kLdThreads];
  __shared__ int lp[kLdThreads];
  const int item = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  int par = 0;
  if (item < nleaf) {
    const int64_t o = leaf_off[item];
    const int m = (int)(leaf_off[item + 1] - o);
    const T* ud = udinv + (int64_t)item * ldl;
    const int32_t* pv = piv + (int64_t)item * ldl;
    for (int j = tid; j < m; j += kLdThreads) {
      const double d = (double)ud[j];  // 1 / U_jj
      s -= log(fabs(d));
      par ^= (d < 0.0) ^ (pv[j] != j);
    }
  } else {
    int k = item - nleaf, p = 0;
    while (p < lv.n && k >= lv.count[p]) k -= lv.count[p++];
    const int n2 = 2 * lv.r[p];
    const T* ud = Kud + lv.kvoff[p] + (int64_t)k * lv.kp[p];
    const int32_t* pv = Kpiv + lv.kvoff[p] + (int64_t)k * lv.kp[p];
    for (int j = tid; j < n2; j += kLdThreads) {
      const double d = (double)ud[j];
      s -= log(fabs(d));
      par ^= (d < 0.0) ^ (pv[j] != j);
    }
    if (tid == 0) par ^= lv.r[p] & 1;  // (-1)^r of the block exchange
  }
  block_sum<kLdThreads>(s, par, ls, lp);
  if (tid == 0) {
    item_log[item] = s;
    item_par[item] = par;
  }
}

__global__ __launch_bounds__(kLdThreads) void logdet_sum_kernel(int nitems, const double* __restrict__ item_log,
                                                                const int* __restrict__ item_par,
                                                                double* __restrict__ out) {
  __shared__ double ls[kLdThreads];
  __shared__ int lp[kLdThreads];
  const int tid = threadIdx.x;
  double s = 0.0;
  int par = 0;
  for (int i = tid; i < nitems; i += kLdThreads) {
    s += item_log[i];
    par ^= item_par[i];
  }
  block_sum<kLdThreads>(s, par, ls, lp);
  if (tid == 0) {
    out[0] = s;
    out[1] = par ? -1.0 : 1.0;
  }
}

template <typename T>
hipError_t launch_logdet(hipStream_t s, int nleaf, int ldl, const int64_t* d_leaf_off, const T* udinv,
                         const int32_t* piv, const T* Kud, const int32_t* Kpiv, const LogdetLevels& lv,
                         double* item_log, int* item_par, double* out) {
  int nitems = nleaf;
  for (int p = 0; p < lv.n; ++p) nitems += lv.count[p];
  hipLaunchKernelGGL(logdet_items_kernel<T>, dim3(nitems), dim3(kLdThreads), 0, s, nleaf, ldl, d_leaf_off, udinv,
                     piv, Kud, Kpiv, lv, item_log, item_par);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(logdet_sum_kernel, dim3(1), dim3(kLdThreads), 0, s, nitems, item_log, item_par, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pieces of the gradient of log|det A| (Jacobi's formula through the
// factorization; the orchestration is in the API):
//   dD_a = D_a^{-T} - Lam(I_a, :) Y(I_a, :)^T
//   dU_m = Lam(I_m, c_l) - Lam(I_m, 1:R_{l-1}) (Y(I_n, 1:R_{l-1})^T V_n)
//   dV_n = Y(I_n, c_l) P_n - Y(I_n, 1:R_{l-1}) (Lam(I_m, 1:R_{l-1})^T U_m)
// for siblings (m, n) at level l with columns c_l, where P_a is the block of
// K_g^{-1} on a's rows and columns (g the parent of a) and
// Lam(I_a, c_l) = A_a^{-T} V_a P_a^T is the level-l block of Y_big of A^T
// times P_a^T.
// ---------------------------------------------------------------------------

// Dt(o + i, j) = D(o + j, i) for the leaf blocks (D_big layout)
template <typename S>
__global__ void transpose_leaves_kernel(const int64_t* __restrict__ leaf_off, int m_max, const S* __restrict__ D,
                                        int64_t ldd, S* __restrict__ Dt, int64_t ldt) {
  const int a = blockIdx.y;
  const int64_t o = leaf_off[a];
  const int m = (int)(leaf_off[a + 1] - o);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m_max * m_max; e += gridDim.x * blockDim.x) {
    const int i = e % m_max, j = e / m_max;
    if (i < m && j < m) Dt[o + i + (int64_t)j * ldt] = D[o + j + (int64_t)i * ldd];
  }
}

// E(o + i, j) = delta_ij for i < m_a, j < ncols (the identity in each leaf's rows)
template <typename T>
__global__ void identity_leaves_kernel(const int64_t* __restrict__ leaf_off, int ncols, T* __restrict__ E,
                                       int64_t lde) {
  const int a = blockIdx.y;
  const int64_t o = leaf_off[a];
  const int m = (int)(leaf_off[a + 1] - o);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * ncols; e += gridDim.x * blockDim.x) {
    const int i = e % m, j = e / m;
    E[o + i + (int64_t)j * lde] = (i == j) ? T(1) : T(0);
  }
}

// nblk stacked n2 x n2 identities: X(g n2 + i, j) = delta_ij, ld = nblk n2
template <typename T>
__global__ void identity_blocks_kernel(int nblk, int n2, T* __restrict__ X) {
  const int64_t ld = (int64_t)nblk * n2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ld * n2; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e % ld;
    const int j = (int)(e / ld);
    X[e] = ((int)(row % n2) == j) ? T(1) : T(0);
  }
}

// P_a for the children a = 2g + h of the parents g of one level: Pd[a][k][c] =
// Kinv_g(h r + k, h r + c), from K^{-1} stored per parent with leading
// dimension ldk and parent stride pstride (elements)
template <typename T>
__global__ void pblocks_kernel(int nparents, int r, const T* __restrict__ Kinv, int64_t ldk, int64_t pstride,
                               double* __restrict__ Pd) {
  const int64_t total = (int64_t)nparents * 2 * r * r;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e / ((int64_t)r * r);
    const int k = (int)((e / r) % r), c = (int)(e % r);
    const int64_t g = a >> 1;
    const int h = (int)(a & 1);
    Pd[e] = (double)Kinv[g * pstride + (h * r + k) + (int64_t)(h * r + c) * ldk];
  }
}

// out(i, c) = sum_k in(i, R_{l-1} + k) M_a(k, c - R_{l-1}) for every column c
// (level l) and row i (node a of level l), M_a = P_a (trans = 0) or P_a^T
// (trans = 1) from Pd at element pdoff[l] + a r_l^2; FP64, N x R, ld N
__global__ void node_mix_kernel(int64_t n, int L, int R, const int64_t* __restrict__ leaf_off,
                                const int32_t* __restrict__ rpre, const int64_t* __restrict__ pdoff,
                                const double* __restrict__ Pd, int trans, const double* __restrict__ in,
                                double* __restrict__ out) {
  const int64_t total = n * R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n;
    const int c = (int)(e / n);
    int l = 1;
    while (l < L && c >= rpre[l]) ++l;
    const int c0 = rpre[l - 1], r = rpre[l] - c0, cc = c - c0;
    // leaf of row i (last leaf offset <= i), then its level-l ancestor
    int lo = 0, hi = 1 << L;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (leaf_off[mid] <= i) lo = mid;
      else hi = mid;
    }
    const int64_t a = lo >> (L - l);
    const double* M = Pd + pdoff[l] + a * r * r;
    double acc = 0.0;
    for (int k = 0; k < r; ++k)
      acc += in[i + (int64_t)(c0 + k) * n] * (trans ? M[cc * r + k] : M[k * r + cc]);
    out[e] = acc;
  }
}

template <typename S>
hipError_t launch_transpose_leaves(hipStream_t s, int nleaf, int m_max, const int64_t* d_leaf_off, const S* D,
                                   int64_t ldd, S* Dt, int64_t ldt) {
  if (nleaf == 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_leaves_kernel<S>, dim3(std::min(64, (m_max * m_max + 255) / 256), nleaf), dim3(256), 0,
                     s, d_leaf_off, m_max, D, ldd, Dt, ldt);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_identity_leaves(hipStream_t s, int nleaf, int ncols, const int64_t* d_leaf_off, T* E, int64_t lde) {
  if (nleaf == 0 || ncols == 0) return hipSuccess;
  hipLaunchKernelGGL(identity_leaves_kernel<T>, dim3(std::min(64, (256 * ncols + 255) / 256), nleaf), dim3(256), 0, s,
                     d_leaf_off, ncols, E, lde);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_identity_blocks(hipStream_t s, int nblk, int n2, T* X) {
  if (nblk == 0 || n2 == 0) return hipSuccess;
  hipLaunchKernelGGL(identity_blocks_kernel<T>, dim3(256), dim3(256), 0, s, nblk, n2, X);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_pblocks(hipStream_t s, int nparents, int r, const T* Kinv, int64_t ldk, int64_t pstride, double* Pd) {
  if (nparents == 0 || r == 0) return hipSuccess;
  hipLaunchKernelGGL(pblocks_kernel<T>, dim3(256), dim3(256), 0, s, nparents, r, Kinv, ldk, pstride, Pd);
  return hipGetLastError();
}
hipError_t launch_node_mix(hipStream_t s, int64_t n, int L, int R, const int64_t* d_leaf_off, const int32_t* d_rpre,
                           const int64_t* d_pdoff, const double* Pd, int trans, const double* in, double* out) {
  if (n == 0 || R == 0) return hipSuccess;
  hipLaunchKernelGGL(node_mix_kernel, dim3(2048), dim3(256), 0, s, n, L, R, d_leaf_off, d_rpre, d_pdoff, Pd, trans, in,
                     out);
  return hipGetLastError();
}
template hipError_t launch_transpose_leaves<double>(hipStream_t, int, int, const int64_t*, const double*, int64_t,
                                                    double*, int64_t);
template hipError_t launch_transpose_leaves<float>(hipStream_t, int, int, const int64_t*, const float*, int64_t,
                                                   float*, int64_t);
template hipError_t launch_identity_leaves<double>(hipStream_t, int, int, const int64_t*, double*, int64_t);
template hipError_t launch_identity_leaves<float>(hipStream_t, int, int, const int64_t*, float*, int64_t);
template hipError_t launch_identity_blocks<double>(hipStream_t, int, int, double*);
template hipError_t launch_identity_blocks<float>(hipStream_t, int, int, float*);
template hipError_t launch_pblocks<double>(hipStream_t, int, int, const double*, int64_t, int64_t, double*);
template hipError_t launch_pblocks<float>(hipStream_t, int, int, const float*, int64_t, int64_t, double*);

template hipError_t launch_logdet<double>(hipStream_t, int, int, const int64_t*, const double*, const int32_t*,
                                          const double*, const int32_t*, const LogdetLevels&, double*, int*, double*);
template hipError_t launch_logdet<float>(hipStream_t, int, int, const int64_t*, const float*, const int32_t*,
                                         const float*, const int32_t*, const LogdetLevels&, double*, int*, double*);

}  // namespace hodlr
