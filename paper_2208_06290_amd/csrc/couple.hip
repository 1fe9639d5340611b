// Coupling systems (Section III-A eq. "e:k"; Alg. "a:gpuf" form K / factor K /
// solve W; Alg. "a:gpus" solve w):
//
//   K_g = [[V_a^T Y_a, I], [I, V_b^T Y_b]]   for the children a, b of parent g
//
// The products V^T Y arrive as per-tile partial sums (level pass) or as
// segment sums of them; they are summed here in fixed order.
//
// couple_factor: one workgroup per parent; K is formed in LDS from the
//   children's reduced products, the right-hand sides
//   [V_a^T Y_big(I_a, 1:R_l); V_b^T Y_big(I_b, 1:R_l)] of eq. "e:node1" are
//   written to W, and K is LU-factored with partial pivoting (largest
//   magnitude, lowest row on ties): by all four waves with K in registers
//   when 2r <= 64, else by one wave in LDS.  The LU of K is stored
//   zero-padded to kp x kp (kp = 2r rounded up to 16) so the block solver
//   needs no bounds checks; couple_dinv then forms the inverted 16 x 16
//   diagonal blocks of L and U, and the MFMA block solver overwrites W with
//   K^{-1} W.
// couple_solve: one wave per parent; w = K^{-1} [V_a^T x_a; V_b^T x_b]
//   (eq. "e:node3") or the transposed solve used by the adjoint.
// Lanes own rows of the right-hand side (2r <= 128 -> two rows per lane) and
// the pivot value of each elimination step is broadcast with readlane.
#include "mfma.h"
#include "wave.h"

#include <algorithm>

namespace hodlr {

// ---------------------------------------------------------------------------
// segment sums: out[s] = sum of tiles [desc[s].x, desc[s].x + desc[s].y)
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ void segment_reduce_kernel(const int2* __restrict__ desc, int64_t elems, const T* __restrict__ P,
                                      T* __restrict__ out) {
  const int sg = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= elems) return;
  const int2 d = desc[sg];  // d.y <= NT items
  // all loads in flight at once (clamped to the segment), summed in item order
  T v[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) v[t] = P[(int64_t)(d.x + min(t, d.y - 1)) * elems + e];
  T acc = v[0];
#pragma unroll
  for (int t = 1; t < NT; ++t)
    if (t < d.y) acc += v[t];
  out[(int64_t)sg * elems + e] = acc;
}

// maxy: largest item count of a segment (<= kSegTiles); the kernel issues that many loads
template <typename T>
hipError_t launch_segment_reduce(hipStream_t s, int nsegs, const int2* d_desc, int64_t elems, const T* P, T* out,
                                 int maxy) {
  if (nsegs == 0 || elems == 0) return hipSuccess;
  if (maxy < 1 || maxy > kSegTiles) return hipErrorInvalidValue;
  dim3 grid((unsigned)((elems + 255) / 256), (unsigned)nsegs);
  if (maxy <= 2)
    hipLaunchKernelGGL((segment_reduce_kernel<T, 2>), grid, dim3(256), 0, s, d_desc, elems, P, out);
  else if (maxy <= 4)
    hipLaunchKernelGGL((segment_reduce_kernel<T, 4>), grid, dim3(256), 0, s, d_desc, elems, P, out);
  else if (maxy <= 8)
    hipLaunchKernelGGL((segment_reduce_kernel<T, 8>), grid, dim3(256), 0, s, d_desc, elems, P, out);
  else
    hipLaunchKernelGGL((segment_reduce_kernel<T, kSegTiles>), grid, dim3(256), 0, s, d_desc, elems, P, out);
  return hipGetLastError();
}
template hipError_t launch_segment_reduce<double>(hipStream_t, int, const int2*, int64_t, const double*, double*, int);
template hipError_t launch_segment_reduce<float>(hipStream_t, int, const int2*, int64_t, const float*, float*, int);

// sum over the segments of `node`: element (i, c) of an r x ncols col-major block
template <typename T>
__device__ __forceinline__ T seg_sum(const T* __restrict__ segs, const int32_t* __restrict__ seg_start, int node,
                                     int64_t elems, int64_t idx) {
  const int s0 = seg_start[node], s1 = seg_start[node + 1];
  T acc = T(0);
  for (int sg = s0; sg < s1; ++sg) acc += segs[(int64_t)sg * elems + idx];
  return acc;
}

template <typename T>
__device__ __forceinline__ T bcast(T v, int srclane);
template <>
__device__ __forceinline__ double bcast<double>(double v, int srclane) {
  int2 u = __builtin_bit_cast(int2, v);
  u.x = __builtin_amdgcn_readlane(u.x, srclane);
  u.y = __builtin_amdgcn_readlane(u.y, srclane);
  return __builtin_bit_cast(double, u);
}
template <>
__device__ __forceinline__ float bcast<float>(float v, int srclane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), srclane));
}

constexpr int kWlsBatch = 16;

// One wave solves K z = y for NC right-hand-side columns held as x[slot][c]
// (row = slot * 64 + lane).  Kf: LU factor (col-major, leading dimension ld),
// kud: reciprocal diagonal.  Rows >= n2 are ignored.
template <typename T, int NC, int TRANS>
__device__ __forceinline__ void wave_lu_solve(T (&x)[2][NC], const T* Kf, const T* kud, int n2, int ld, int lane) {
  // The factor entries a step needs do not depend on x: they are loaded
  // kWlsBatch steps at a time (one memory latency per batch instead of per
  // step); rows past n2 load a clamped row and are never used.
  constexpr int B = kWlsBatch;
  const int rr[2] = {lane, min(64 + lane, n2 - 1)};
  auto step_lower = [&](int j, const T (&f)[2]) {  // x(rows > j) -= f x_j (unit diagonal)
    const int sj = j >> 6, lj = j & 63;
    T xj[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xj[c] = bcast(sj ? x[1][c] : x[0][c], lj);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int row = s * 64 + lane;
      if (row > j && row < n2) {
#pragma unroll
        for (int c = 0; c < NC; ++c) x[s][c] -= f[s] * xj[c];
      }
    }
  };
  auto step_upper = [&](int j, const T (&f)[2], T dinv, bool below) {  // x_j *= 1/d_j; x(rows beyond j) -= f x_j
    const int sj = j >> 6, lj = j & 63;
    T xj[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xj[c] = bcast(sj ? x[1][c] : x[0][c], lj) * dinv;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int row = s * 64 + lane;
      if (row == j) {
#pragma unroll
        for (int c = 0; c < NC; ++c) x[s][c] = xj[c];
      } else if (below ? (row > j && row < n2) : (row < j)) {
#pragma unroll
        for (int c = 0; c < NC; ++c) x[s][c] -= f[s] * xj[c];
      }
    }
  };
  auto step_lower_back = [&](int j, const T (&f)[2]) {  // x(rows < j) -= f x_j (unit diagonal)
    const int sj = j >> 6, lj = j & 63;
    T xj[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xj[c] = bcast(sj ? x[1][c] : x[0][c], lj);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int row = s * 64 + lane;
      if (row < j) {
#pragma unroll
        for (int c = 0; c < NC; ++c) x[s][c] -= f[s] * xj[c];
      }
    }
  };
  // f[q][s] = entry (row s, step j0 + q): column j of the factor (colmajor) or row j (transposed)
  auto load = [&](int j0, T (&f)[B][2], T (&dv)[B], bool colmajor, int dir) {
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int j = min(max(j0 + dir * q, 0), n2 - 1);
#pragma unroll
      for (int s = 0; s < 2; ++s) f[q][s] = colmajor ? Kf[rr[s] + (int64_t)j * ld] : Kf[j + (int64_t)rr[s] * ld];
      dv[q] = kud[j];
    }
  };
  T f[B][2], dv[B];
  if (!TRANS) {
    // L (unit lower) then U
    for (int j0 = 0; j0 < n2; j0 += B) {
      load(j0, f, dv, true, 1);
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (j0 + q < n2) step_lower(j0 + q, f[q]);
    }
    for (int j0 = n2 - 1; j0 >= 0; j0 -= B) {
      load(j0, f, dv, true, -1);
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (j0 - q >= 0) step_upper(j0 - q, f[q], dv[q], false);
    }
  } else {
    // U^T (lower, non-unit) then L^T (unit upper)
    for (int j0 = 0; j0 < n2; j0 += B) {
      load(j0, f, dv, false, 1);
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (j0 + q < n2) step_upper(j0 + q, f[q], dv[q], true);
    }
    for (int j0 = n2 - 1; j0 >= 0; j0 -= B) {
      load(j0, f, dv, false, -1);
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (j0 - q >= 0) step_lower_back(j0 - q, f[q]);
    }
  }
}

// ---------------------------------------------------------------------------
// couple_factor
// ---------------------------------------------------------------------------
constexpr int kCfThreads = 256;

// LU with partial pivoting of the n2 x n2 (n2 <= 64) matrix K (LDS, col-major)
// by the four waves of the workgroup with the matrix in registers: lane i
// holds row i, wave w columns 16w .. 16w+15.  Rows are not moved while
// factoring; each lane tracks the position of its row.  At step j the wave
// owning column j picks the largest |K(., j)| among unpivoted rows (lowest
// position on ties, a NaN counts as infinite) and publishes the multipliers
// through LDS (double buffered: one barrier per step); every wave then takes
// the pivot row from its own registers with readlane and updates its columns.
// Steps run in blocks of 16 (the owner's column is then a compile-time
// register index); a wave whose columns all lie left of the current block
// has nothing to update, a wave right of it updates all 16 columns without
// per-column tests.  On return K holds L\U in pivoted order, spiv[j] the
// LAPACK-style interchange of step j and sperm[i] the original row at
// position i.
template <typename T>
__device__ __forceinline__ void block_lu(T* K, int n2, int lane, int w, int* spiv, int* sperm,
                                         unsigned long long* info, unsigned long long info_base) {
  __shared__ T s_l[2][64];
  __shared__ int s_pl[2][2];  // pivot lane, pivot value nonzero
  T kc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = 16 * w + c;
    kc[c] = (lane < n2 && col < n2) ? K[lane + col * n2] : T(0);
  }
  int mypos = lane;
  bool done = lane >= n2;
  const int nb = (n2 + 15) >> 4;
  for (int jb = 0; jb < nb; ++jb) {
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * jb + jj;
      if (j < n2) {  // uniform
        const int sb = jj & 1;
        if (w == jb) {
          const T kj = kc[jj];
          T v = done ? T(-1) : fabs(kj);
          if (!done && !(v == v)) v = T(INFINITY);
          T vmax;
          int bk;  // pivot position (uniform)
          wave_argmax(v, done ? 0x7fffffff : mypos, vmax, bk);
          const unsigned long long sel = __ballot(!done && mypos == bk);
          const int plane = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(sel));
          const T pv = bcast(kj, plane);
          const bool nz = pv != T(0);
          s_l[sb][lane] = (!done && lane != plane && nz) ? kj * (T(1) / pv) : T(0);
          if (lane == 0) {
            s_pl[sb][0] = plane;
            s_pl[sb][1] = nz;
            spiv[j] = bk;
            if (!nz) atomicMin(info, info_base | (unsigned long long)j);
          }
        }
        __syncthreads();
        const int plane = __builtin_amdgcn_readfirstlane(s_pl[sb][0]);
        const bool nz = s_pl[sb][1] != 0;
        const T l = s_l[sb][lane];
        const bool me = lane == plane;
        const bool upd = !done && !me && nz;
        const int bk = __builtin_amdgcn_readfirstlane(__shfl(mypos, plane, 64));
        if (!done && !me && mypos == j) mypos = bk;  // the row displaced by the interchange
        if (me) {
          done = true;
          mypos = j;
        }
        if (w == jb) {
          kc[jj] = upd ? l : kc[jj];
#pragma unroll
          for (int c = jj + 1; c < 16; ++c) {
            const T pc = bcast(kc[c], plane);
            kc[c] = upd ? kc[c] - l * pc : kc[c];
          }
        } else if (w > jb) {
#pragma unroll
          for (int c = 0; c < 16; ++c) {
            const T pc = bcast(kc[c], plane);
            kc[c] = upd ? kc[c] - l * pc : kc[c];
          }
        }
      }
    }
  }
  __syncthreads();  // every wave has read K before it is overwritten
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = 16 * w + c;
    if (lane < n2 && col < n2) K[mypos + col * n2] = kc[c];
  }
  if (w == 0 && lane < n2) sperm[mypos] = lane;
}

// K_g (eq. "e:k") in LDS, col-major n2 x n2, from the children's reduced
// products: item columns Rp .. Rp + r - 1 hold V_a^T Y_a (r x r)
template <typename T>
__device__ __forceinline__ void form_k(T* K, const T* Pa, const T* Pb, int r, int Rp, int tid) {
  const int n2 = 2 * r;
#pragma unroll 4
  for (int e = tid; e < n2 * n2; e += kCfThreads) {
    const int i = e % n2, j = e / n2;
    const bool da = i < r && j < r, db = i >= r && j >= r;
    const T va = Pa[min(i, r - 1) + (int64_t)(Rp + min(j, r - 1)) * r];
    const T vb = Pb[max(i - r, 0) + (int64_t)(Rp + max(j - r, 0)) * r];
    const T id = (i < r ? j - r == i : i - r == j) ? T(1) : T(0);
    K[i + j * n2] = da ? va : (db ? vb : id);
  }
}

// Element e = tid + u * NT (u = 0, 1, ...) of an n2-row column-major block as
// (row, column), stepped without a division per element.
struct BlockWalk {
  int k, c, dq, dr, n2;
  __device__ __forceinline__ BlockWalk(int tid, int nt, int n2_) : n2(n2_) {
    k = tid % n2;
    c = tid / n2;
    dq = nt / n2;
    dr = nt % n2;
  }
  __device__ __forceinline__ void next() {
    k += dr;
    c += dq;
    if (k >= n2) {
      k -= n2;
      ++c;
    }
  }
};

// form_k for the inverse route (n2 * n2 <= NT * NPT): every thread issues its
// NPT loads in batches of NB, each entry read from the one product it comes
// from
template <typename T, int NT, int NPT, int NB>
__device__ __forceinline__ void form_k_batched(T* K, const T* Pa, const T* Pb, int r, int Rp, int tid) {
  static_assert(NPT % NB == 0, "whole batches");
  const int n2 = 2 * r;
  asm volatile("" : "+v"(tid));
  BlockWalk it(tid, NT, n2);
  for (int u0 = 0; u0 < NPT; u0 += NB) {
    T v[NB];
    BlockWalk st = it;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int i = it.k, j = it.c;
      T x = (i < r ? j - r == i : i - r == j) ? T(1) : T(0);
      if (j < n2) {
        if (i < r && j < r) x = Pa[i + (int64_t)(Rp + j) * r];
        else if (i >= r && j >= r) x = Pb[(i - r) + (int64_t)(Rp + j - r) * r];
      }
      v[u] = x;
      it.next();
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (st.c < n2) K[st.k + st.c * n2] = v[u];
      st.next();
    }
  }
}

// One 64-column chunk of the right-hand sides [W_a; W_b] (columns c0 ..
// c0 + 63 of the children's products, zero past Rp): NPT values per thread
// loaded in one batch (64 * n2 <= NT * NPT), then stored to LDS as
// [column][row] with ld n2 + 1.
template <typename T, int NT, int NPT>
struct RhsChunk {
  T v[NPT];
  __device__ __forceinline__ void load(const T* Pa, const T* Pb, int r, int Rp, int c0, int tid) {
    // an opaque copy of tid: the per-element addresses are not hoisted out of
    // the caller's chunk loop (they would stay live in registers)
    asm volatile("" : "+v"(tid));
    BlockWalk it(tid, NT, 2 * r);
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const int k = it.k, col = c0 + it.c;
      T x = T(0);
      if (it.c < 64 && col < Rp) x = k < r ? Pa[k + (int64_t)col * r] : Pb[(k - r) + (int64_t)col * r];
      v[u] = x;
      it.next();
    }
  }
  __device__ __forceinline__ void store(T* Rs, int r, int tid) const {
    const int n2 = 2 * r, ldr = n2 + 1;
    BlockWalk it(tid, NT, n2);
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      if (it.c < 64) Rs[it.c * ldr + it.k] = v[u];
      it.next();
    }
  }
};

// Gauss-Jordan elimination with partial pivoting on [K | I] for n2 <= 64,
// n2 % 16 == 0, with the same register layout and pivot rule as block_lu
// (lane i holds row i, wave w columns 16w .. 16w+15 of K and of the augmented
// block).  Step j eliminates column j from every other row, including the
// rows pivoted earlier.  The pivot rows are divided by their pivots only at
// the end (a row scaled later is the same multiple of the row scaled at once
// through every later elimination, which is linear in it), so each step is
// one multiply-add per entry; rows not yet pivoted are not affected, so the
// pivots are those of scaling at once.  Afterwards the augmented row of the
// row pivoted at step j, divided by its pivot, is row j of K^{-1}, written to
// K (col-major).
// spiv[j] records the position the row pivoted at step j came from (an
// interchange with position j, as LAPACK's ipiv) and spv[j] its pivot value:
// the pivots are those of LU with partial pivoting, so they give det K.
template <typename T>
__device__ __forceinline__ void block_gj(T* K, int n2, int lane, int w, int* spiv, T* spv, unsigned long long* info,
                                         unsigned long long info_base) {
  __shared__ T s_l[2][64];
  __shared__ int s_pl[2][2];  // pivot lane, pivot position
  T kc[16], ac[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = 16 * w + c;
    kc[c] = (lane < n2 && col < n2) ? K[lane + col * n2] : T(0);
    ac[c] = (lane < n2 && lane == col) ? T(1) : T(0);
  }
  int mypos = lane;
  bool done = lane >= n2;
  const int nb = n2 >> 4;
  // pivot search of column j (value kj of the lane's row), by the wave that
  // owns the column: the multipliers and the pivot go to slot sb
  auto pivot = [&](int j, T kj, int sb) {
    T v = done ? T(-1) : fabs(kj);
    if (!done && !(v == v)) v = T(INFINITY);
    T vmax;
    int bk;  // pivot position (uniform)
    wave_argmax(v, done ? 0x7fffffff : mypos, vmax, bk);
    const unsigned long long sel = __ballot(!done && mypos == bk);
    const int plane = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(sel));
    const T pv = bcast(kj, plane);
    const bool nz = pv != T(0);
    const T rp = T(1) / pv;
    // multipliers of the other rows; the pivot row keeps its values (scaled at the end)
    s_l[sb][lane] = (lane < n2 && nz && lane != plane) ? kj * rp : T(0);
    if (lane == 0) {
      s_pl[sb][0] = plane;
      s_pl[sb][1] = bk;
      spiv[j] = bk;
      spv[j] = pv;
      if (!nz) atomicMin(info, info_base | (unsigned long long)j);
    }
  };
  for (int jb = 0; jb < nb; ++jb) {
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * jb + jj;
      const int sb = jj & 1;
      // the first column of a block; the others were searched ahead (below)
      if (jj == 0 && w == jb) pivot(j, kc[0], sb);
      __syncthreads();
      // after a zero pivot (reported) every multiplier is zero and the rows
      // stay as they are
      const int plane = __builtin_amdgcn_readfirstlane(s_pl[sb][0]);
      const int bk = __builtin_amdgcn_readfirstlane(s_pl[sb][1]);
      const T l = s_l[sb][lane];
      const bool me = lane == plane;
      if (!done && !me && mypos == j) mypos = bk;  // the row displaced by the interchange
      if (me) {
        done = true;
        mypos = j;
      }
      auto elim = [&](T& x) {
        const T p = bcast(x, plane);
        x = x - l * p;  // l = 0 in the pivot row
      };
      // columns left of j are zero in the pivot row: nothing to do there.
      // The owner eliminates column j + 1 first and searches its pivot
      // before the rest of its work, so that search is off the other waves'
      // critical path.
      if (w == jb) {
        if (jj < 15) {
          elim(kc[jj + 1]);
          pivot(j + 1, kc[jj + 1], sb ^ 1);
        }
#pragma unroll
        for (int c = jj + 2; c < 16; ++c) elim(kc[c]);
      } else if (w > jb) {
#pragma unroll
        for (int c = 0; c < 16; ++c) elim(kc[c]);
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) elim(ac[c]);
    }
  }
  __syncthreads();  // every wave has read K before it is overwritten
  // the row pivoted at step mypos, divided by its pivot (left as it is after a
  // zero pivot, which is reported)
  const T pvm = lane < n2 ? spv[mypos] : T(1);
  const T sc = pvm != T(0) ? T(1) / pvm : T(1);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = 16 * w + c;
    if (lane < n2 && col < n2) K[mypos + col * n2] = ac[c] * sc;
  }
}

template <typename T>
__global__ __launch_bounds__(kCfThreads) void couple_factor_kernel(int r, int kp, int Rp, const T* __restrict__ segs,
                                                                   const int32_t* __restrict__ seg_start,
                                                                   T* __restrict__ Klu, int32_t* __restrict__ Kpiv,
                                                                   int32_t* __restrict__ Kperm,
                                                                   T* __restrict__ Kud,
                                                                   T* __restrict__ W, unsigned long long* info,
                                                                   int level, int L) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* K = reinterpret_cast<T*>(smem_raw);  // n2 x n2, col-major
  __shared__ int spiv[2 * HODLR_MAX_RANK];
  __shared__ int sperm[2 * HODLR_MAX_RANK];

  const int g = blockIdx.x;
  const int a = 2 * g, b = 2 * g + 1;
  const int n2 = 2 * r;
  const int ncin = Rp + r;  // columns of the children's products: [W rhs | T]
  const int64_t elems = (int64_t)r * ncin;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  // the children's products have been reduced to one item per node
  const T* Pa = segs + (int64_t)seg_start[a] * elems;
  const T* Pb = segs + (int64_t)seg_start[b] * elems;
  form_k(K, Pa, Pb, r, Rp, tid);
  __syncthreads();
  // right-hand sides of eq. "e:node1", unpermuted (the block solver applies the pivots)
  {
    T* Wg = W + (int64_t)g * n2 * Rp;
#pragma unroll 4
    for (int e = tid; e < n2 * Rp; e += kCfThreads) {
      const int i = e % n2, cc = e / n2;
      Wg[e] = (i < r ? Pa : Pb)[(i % r) + (int64_t)cc * r];
    }
  }
  if (n2 <= 64) {
    block_lu(K, n2, lane, wid, spiv, sperm, info, ((unsigned long long)(L - level) << 44) | ((unsigned long long)g << 16));
  } else {
    // LU with partial pivoting, 64 < 2r <= 128: per column, wave 0 takes the
    // pivot (rows over lanes, two rows a lane), exchanges the rows and scales
    // the column below the pivot; then the four waves update the trailing
    // columns, wave w the columns c = w (mod 4) right of j.  Every entry gets
    // the same operations in the same order as in a sequential elimination.
    __shared__ T lcol[2 * HODLR_MAX_RANK];
    __shared__ T prow[2 * HODLR_MAX_RANK];
    __shared__ int zero_pivot;
    for (int j = 0; j < n2; ++j) {
      if (wid == 0) {
        T best = T(-1);
        int bi = 0x7fffffff;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int row = sl * 64 + lane;
          if (row >= j && row < n2) {
            T v = fabs(K[row + j * n2]);
            if (!(v == v)) v = T(INFINITY);
            if (v > best || (v == best && row < bi)) {
              best = v;
              bi = row;
            }
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const T ov = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ov > best || (ov == best && oi < bi)) {
            best = ov;
            bi = oi;
          }
        }
        const int p = (bi < n2) ? bi : j;
        if (lane == 0) {
          spiv[j] = p;
          if (K[p + j * n2] == T(0))
            atomicMin(info, ((unsigned long long)(L - level) << 44) | ((unsigned long long)g << 16) |
                                (unsigned long long)j);
        }
        if (p != j) {
#pragma unroll
          for (int sl = 0; sl < 2; ++sl) {
            const int c = sl * 64 + lane;
            if (c < n2) {
              const T t0 = K[j + c * n2];
              K[j + c * n2] = K[p + c * n2];
              K[p + c * n2] = t0;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const T pivot = K[j + j * n2];
        const T rinv = pivot != T(0) ? T(1) / pivot : T(0);
        if (lane == 0) zero_pivot = pivot == T(0);  // no elimination step then
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int row = sl * 64 + lane;
          if (row < n2) {
            // the multipliers below the pivot (zero when the pivot is zero: no update)
            const T l = row > j ? K[row + j * n2] * rinv : T(0);
            lcol[row] = l;
            if (row > j && pivot != T(0)) K[row + j * n2] = l;
            prow[row] = K[j + row * n2];  // the pivot row (entry c at prow[c])
          }
        }
      }
      __syncthreads();
      if (!zero_pivot) {
        // four of the wave's columns per round, their loads issued together
        // (rows past n2 read a clamped row and write nothing)
        const int r0 = lane, r1 = min(64 + lane, n2 - 1);
        const bool w0 = r0 > j && r0 < n2, w1 = 64 + lane > j && 64 + lane < n2;
        const T l0 = lcol[r0], l1 = lcol[r1];
        int c = j + 1 + wid;
        for (; c + 12 < n2; c += 16) {
          T a[4], b[4], pc[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            pc[q] = prow[c + 4 * q];
            a[q] = K[r0 + (c + 4 * q) * n2];
            b[q] = K[r1 + (c + 4 * q) * n2];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (w0) K[r0 + (c + 4 * q) * n2] = a[q] - l0 * pc[q];
            if (w1) K[r1 + (c + 4 * q) * n2] = b[q] - l1 * pc[q];
          }
        }
        for (; c < n2; c += 4) {
          const T pc = prow[c];
          const T a = K[r0 + c * n2], b = K[r1 + c * n2];
          if (w0) K[r0 + c * n2] = a - l0 * pc;
          if (w1) K[r1 + c * n2] = b - l1 * pc;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // store the factors (zero-padded kp x kp), the composed permutation and the reciprocal diagonal
  T* Kg = Klu + (int64_t)g * kp * kp;
  for (int e = tid; e < kp * kp; e += kCfThreads) {
    const int i = e % kp, j = e / kp;
    Kg[e] = (i < n2 && j < n2) ? K[i + j * n2] : T(0);
  }
  if (n2 > 64 && tid == 0) {  // (block_lu records the row order itself)
    for (int i = 0; i < n2; ++i) sperm[i] = i;
    for (int j = 0; j < n2; ++j) {
      int p = spiv[j];
      int t0 = sperm[j];
      sperm[j] = sperm[p];
      sperm[p] = t0;
    }
  }
  __syncthreads();
  for (int i = tid; i < kp; i += kCfThreads) {
    Kpiv[(int64_t)g * kp + i] = i < n2 ? spiv[i] : i;
    Kperm[(int64_t)g * kp + i] = i < n2 ? sperm[i] : i;
    Kud[(int64_t)g * kp + i] = i < n2 ? T(1) / K[i + i * n2] : T(1);
  }
}

// Inverses of the 16 x 16 diagonal blocks of L and U of every factored K
// (padded part: identity), for the block solver.  A kernel of its own: the
// unrolled substitutions need many registers, which would cap the occupancy of
// the factorization.  Thread (which, kb, cc) forms column cc of block kb.
template <typename T>
__global__ __launch_bounds__(kCfThreads) void couple_dinv_kernel(int n2, int kp, const T* __restrict__ Klu,
                                                                 T* __restrict__ Kinv) {
  const int g = blockIdx.x, tid = threadIdx.x;
  const int nbd = kp >> 4;
  const int which = tid >> 7;  // 0: L, 1: U
  const int kb = (tid >> 4) & 7, cc = tid & 15;
  if (kb >= nbd) return;
  const int g0 = 16 * kb;
  const T* Kg = Klu + (int64_t)g * kp * kp + g0 + (int64_t)g0 * kp;  // zero-padded kp x kp, col-major
  auto Kel = [&](int i, int j) -> T { return Kg[i + j * kp]; };
  T x[16];
  if (which == 0) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      T sv = (i == cc) ? T(1) : T(0);
#pragma unroll
      for (int jj = 0; jj < i; ++jj) sv -= Kel(i, jj) * x[jj];
      x[i] = (i >= cc) ? sv : T(0);
    }
  } else {
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      T sv = (i == cc) ? T(1) : T(0);
#pragma unroll
      for (int jj = i + 1; jj < 16; ++jj) sv -= Kel(i, jj) * x[jj];
      const T d = (g0 + i < n2) ? Kel(i, i) : T(1);
      x[i] = (i <= cc) ? sv / d : T(0);
    }
  }
  T* dst = Kinv + ((int64_t)g * 2 + which) * nbd * 256 + kb * 256;
#pragma unroll
  for (int i = 0; i < 16; ++i) dst[i * 16 + cc] = x[i];
}

// Coupling factor for 2r <= 64, 2r % 16 == 0: K^{-1} by block_gj, stored
// (2r x 2r, col-major) for the solves, and W = K^{-1} rhs written directly:
// the products run on MFMA in 64-column chunks, transposed
// (W^T = rhs^T K^{-T}) so that lanes hold consecutive rows of W; wave w forms
// rows 16w .. 16w+15 with its part of K^{-1} held in registers, and the
// right-hand-side chunk is staged in LDS (where K was).
template <typename T>
__global__ __launch_bounds__(kCfThreads) void couple_factor_inv_kernel(int r, int Rp, const T* __restrict__ segs,
                                                                       const int32_t* __restrict__ seg_start,
                                                                       T* __restrict__ Kinv, int32_t* __restrict__ Kpiv,
                                                                       T* __restrict__ Kud, T* __restrict__ W,
                                                                       unsigned long long* info, int level, int L) {
  using M = Mfma<T>;
  using V = typename M::V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* K = reinterpret_cast<T*>(smem_raw);  // n2 x n2 col-major, then the rhs chunk [c][k] (ld n2 + 1)
  const int g = blockIdx.x;
  const int a = 2 * g, b = 2 * g + 1;
  const int n2 = 2 * r;
  const int ncin = Rp + r;
  const int64_t elems = (int64_t)r * ncin;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lq = lane >> 4;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const T* Pa = segs + (int64_t)seg_start[a] * elems;
  const T* Pb = segs + (int64_t)seg_start[b] * elems;
  __shared__ int s_piv[64];
  __shared__ T s_pv[64];
  form_k_batched<T, kCfThreads, 16, 8>(K, Pa, Pb, r, Rp, tid);
  __syncthreads();
  block_gj(K, n2, lane, wid, s_piv, s_pv, info, ((unsigned long long)(L - level) << 44) | ((unsigned long long)g << 16));
  __syncthreads();
  T* Kg = Kinv + (int64_t)g * n2 * n2;
  for (int e = tid; e < n2 * n2; e += kCfThreads) Kg[e] = K[e];
  // interchanges and reciprocal pivots, as the LU route stores them (for det K)
  if (tid < n2) {
    Kpiv[(int64_t)g * n2 + tid] = s_piv[tid];
    Kud[(int64_t)g * n2 + tid] = T(1) / s_pv[tid];
  }
  // B operand: K^{-1}(16 wid + li, 4 ks + lq)
  const bool act = 16 * wid < n2;  // uniform
  T bk[16];
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) bk[ks] = (act && 4 * ks < n2) ? K[(16 * wid + li) + (4 * ks + lq) * n2] : T(0);
  __syncthreads();  // K's LDS is reused for the right-hand sides
  T* Rs = K;
  const int ldr = n2 + 1;
  T* Wg = W + (int64_t)g * n2 * Rp;
  for (int c0 = 0; c0 < Rp; c0 += 64) {
    {
      RhsChunk<T, kCfThreads, 16> rhs;
      rhs.load(Pa, Pb, r, Rp, c0, tid);
      rhs.store(Rs, r, tid);
    }
    __syncthreads();
    if (act) {
      V acc[4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) acc[mb] = vzero<V>();
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        if (4 * ks < n2) {  // uniform
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) acc[mb] = M::mma(Rs[(16 * mb + li) * ldr + 4 * ks + lq], bk[ks], acc[mb]);
        }
      }
      const int i = 16 * wid + li;
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = c0 + 16 * mb + M::crow(lq, t);
          if (c < Rp) Wg[i + (int64_t)c * n2] = acc[mb][t];
        }
    }
    __syncthreads();
  }
}

// Gauss-Jordan elimination as block_gj for 64 < n2 <= 128 (n2 % 16 == 0):
// eight waves, wave w holding columns 16w .. 16w+15 of K and of the
// augmented block, lane i holding rows i (slot 0) and 64 + i (slot 1).  The
// pivot of column j is the largest modulus among the rows not pivoted yet,
// the lowest current position on ties (the rule of LU with partial
// pivoting); spiv / spv, the deferred scaling of the pivot rows and their
// final placement as block_gj.
template <typename T>
__device__ __forceinline__ void block_gj2(T* K, int n2, int lane, int w, int* spiv, T* spv, unsigned long long* info,
                                          unsigned long long info_base) {
  __shared__ T s_l[2][128];
  __shared__ int s_pl[2][3];  // pivot lane, pivot slot, pivot position
  T kc[2][16], ac[2][16];
#pragma unroll
  for (int sl = 0; sl < 2; ++sl)
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int row = 64 * sl + lane, col = 16 * w + c;
      kc[sl][c] = (row < n2 && col < n2) ? K[row + col * n2] : T(0);
      ac[sl][c] = (row < n2 && row == col) ? T(1) : T(0);
    }
  int mypos[2] = {lane, 64 + lane};
  bool done[2] = {lane >= n2, 64 + lane >= n2};
  const int nb = n2 >> 4;
  // pivot search of column j (values k0, k1 of the lane's two rows), by the
  // wave that owns the column: multipliers and pivot to slot sb
  auto pivot = [&](int j, T k0, T k1, int sb) {
    const T kj[2] = {k0, k1};
    T v[2];
    int key[2];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      T a = fabs(kj[sl]);
      if (!(a == a)) a = T(INFINITY);
      v[sl] = done[sl] ? T(-1) : a;
      key[sl] = done[sl] ? 0x7fffffff : mypos[sl];
    }
    const int bs = (v[1] > v[0] || (v[1] == v[0] && key[1] < key[0])) ? 1 : 0;
    const T vb = bs ? v[1] : v[0];
    const int kb = bs ? key[1] : key[0];
    T vmax;
    int bk;  // position of the pivot row (uniform)
    wave_argmax(vb, kb, vmax, bk);
    const unsigned long long sel = __ballot(kb == bk);  // positions of rows not pivoted are distinct
    const int plane = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(sel));
    const int pslot = __builtin_amdgcn_readlane(bs, plane);
    const T pv = bcast(pslot ? kj[1] : kj[0], plane);
    const bool nz = pv != T(0);
    const T rp = T(1) / pv;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int row = 64 * sl + lane;
      if (row < n2) s_l[sb][row] = (nz && !(lane == plane && sl == pslot)) ? kj[sl] * rp : T(0);
    }
    if (lane == 0) {
      s_pl[sb][0] = plane;
      s_pl[sb][1] = pslot;
      s_pl[sb][2] = bk;
      spiv[j] = bk;
      spv[j] = pv;
      if (!nz) atomicMin(info, info_base | (unsigned long long)j);
    }
  };
  for (int jb = 0; jb < nb; ++jb) {
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * jb + jj;
      const int sb = jj & 1;
      // the first column of a block; the others were searched ahead (below)
      if (jj == 0 && w == jb) pivot(j, kc[0][0], kc[1][0], sb);
      __syncthreads();
      // after a zero pivot (reported) every multiplier is zero and the rows
      // stay as they are
      const int plane = __builtin_amdgcn_readfirstlane(s_pl[sb][0]);
      const int pslot = __builtin_amdgcn_readfirstlane(s_pl[sb][1]);
      const int bk = __builtin_amdgcn_readfirstlane(s_pl[sb][2]);
      T l[2];
      bool me[2];
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        l[sl] = s_l[sb][min(64 * sl + lane, n2 - 1)];
        me[sl] = lane == plane && sl == pslot;
      }
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        if (!done[sl] && !me[sl] && mypos[sl] == j) mypos[sl] = bk;  // the row displaced by the interchange
        if (me[sl]) {
          done[sl] = true;
          mypos[sl] = j;
        }
      }
      auto elim_col = [&](T (&m)[2][16], int c) {
        const T p = bcast(pslot ? m[1][c] : m[0][c], plane);
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) m[sl][c] = m[sl][c] - l[sl] * p;  // l = 0 in the pivot row
      };
      // the owner eliminates column j + 1 first and searches its pivot
      // before the rest of its work
      if (w == jb) {
        if (jj < 15) {
          elim_col(kc, jj + 1);
          pivot(j + 1, kc[0][jj + 1], kc[1][jj + 1], sb ^ 1);
        }
#pragma unroll
        for (int c = jj + 2; c < 16; ++c) elim_col(kc, c);
      } else if (w > jb) {
#pragma unroll
        for (int c = 0; c < 16; ++c) elim_col(kc, c);
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) elim_col(ac, c);
    }
  }
  __syncthreads();  // every wave has read K before it is overwritten
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int row = 64 * sl + lane;
    const T pvm = row < n2 ? spv[mypos[sl]] : T(1);
    const T sc = pvm != T(0) ? T(1) / pvm : T(1);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int col = 16 * w + c;
      if (row < n2 && col < n2) K[mypos[sl] + col * n2] = ac[sl][c] * sc;
    }
  }
}

// Coupling factor for 64 < 2r <= 128 (2r % 16 == 0): K^{-1} by block_gj2 with
// eight waves, stored (2r x 2r, col-major), and W = K^{-1} rhs on MFMA
// (transposed, as couple_factor_inv_kernel): wave w forms rows 16w .. 16w+15.
constexpr int kCf2Threads = 512;
template <typename T>
__global__ __launch_bounds__(kCf2Threads) void couple_factor_inv2_kernel(int r, int Rp, const T* __restrict__ segs,
                                                                         const int32_t* __restrict__ seg_start,
                                                                         T* __restrict__ Kinv,
                                                                         int32_t* __restrict__ Kpiv,
                                                                         T* __restrict__ Kud, T* __restrict__ W,
                                                                         unsigned long long* info, int level, int L) {
  using M = Mfma<T>;
  using V = typename M::V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* K = reinterpret_cast<T*>(smem_raw);  // n2 x n2 col-major, then the rhs chunk [c][k] (ld n2 + 1)
  const int g = blockIdx.x;
  const int a = 2 * g, b = 2 * g + 1;
  const int n2 = 2 * r;
  const int ncin = Rp + r;
  const int64_t elems = (int64_t)r * ncin;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lq = lane >> 4;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const T* Pa = segs + (int64_t)seg_start[a] * elems;
  const T* Pb = segs + (int64_t)seg_start[b] * elems;
  __shared__ int s_piv[128];
  __shared__ T s_pv[128];
  form_k_batched<T, kCf2Threads, 32, 8>(K, Pa, Pb, r, Rp, tid);
  __syncthreads();
  block_gj2(K, n2, lane, wid, s_piv, s_pv, info, ((unsigned long long)(L - level) << 44) | ((unsigned long long)g << 16));
  __syncthreads();
  T* Kg = Kinv + (int64_t)g * n2 * n2;
  for (int e = tid; e < n2 * n2; e += kCf2Threads) Kg[e] = K[e];
  if (tid < n2) {
    Kpiv[(int64_t)g * n2 + tid] = s_piv[tid];
    Kud[(int64_t)g * n2 + tid] = T(1) / s_pv[tid];
  }
  // B operand: K^{-1}(16 wid + li, 4 ks + lq)
  const bool act = 16 * wid < n2;  // uniform
  T bk[32];
#pragma unroll
  for (int ks = 0; ks < 32; ++ks) bk[ks] = (act && 4 * ks < n2) ? K[(16 * wid + li) + (4 * ks + lq) * n2] : T(0);
  __syncthreads();  // K's LDS is reused for the right-hand sides
  T* Rs = K;
  const int ldr = n2 + 1;
  T* Wg = W + (int64_t)g * n2 * Rp;
  for (int c0 = 0; c0 < Rp; c0 += 64) {
    {
      RhsChunk<T, kCf2Threads, 16> rhs;
      rhs.load(Pa, Pb, r, Rp, c0, tid);
      rhs.store(Rs, r, tid);
    }
    __syncthreads();
    if (act) {
      V acc[4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) acc[mb] = vzero<V>();
#pragma unroll
      for (int ks = 0; ks < 32; ++ks) {
        if (4 * ks < n2) {  // uniform
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) acc[mb] = M::mma(Rs[(16 * mb + li) * ldr + 4 * ks + lq], bk[ks], acc[mb]);
        }
      }
      const int i = 16 * wid + li;
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = c0 + 16 * mb + M::crow(lq, t);
          if (c < Rp) Wg[i + (int64_t)c * n2] = acc[mb][t];
        }
    }
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_couple_factor(hipStream_t s, int nparents, int r, int kp, int Rp, const T* segs,
                                const int32_t* d_seg_start, T* Klu, int32_t* Kpiv, int32_t* Kperm, T* Kud, T* Kinv,
                                T* W, unsigned long long* info, int level, int L) {
  if (nparents == 0 || r == 0) return hipSuccess;
  if (kp > 128) return hipErrorInvalidValue;
  if (couple_uses_inverse(r) && 2 * r > 64) {
    const size_t smem_inv = sizeof(T) * std::max<size_t>((size_t)4 * r * r, (size_t)64 * (2 * r + 1));
    auto ki = couple_factor_inv2_kernel<T>;
    hipError_t e = hipFuncSetAttribute((const void*)ki, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_inv);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ki, dim3(nparents), dim3(kCf2Threads), smem_inv, s, r, Rp, segs, d_seg_start, Klu, Kpiv, Kud, W,
                       info, level, L);
    return hipGetLastError();
  }
  if (couple_uses_inverse(r)) {
    const size_t smem_inv = sizeof(T) * std::max<size_t>((size_t)4 * r * r, (size_t)64 * (2 * r + 1));
    auto ki = couple_factor_inv_kernel<T>;
    hipError_t e = hipFuncSetAttribute((const void*)ki, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_inv);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ki, dim3(nparents), dim3(kCfThreads), smem_inv, s, r, Rp, segs, d_seg_start, Klu, Kpiv, Kud, W,
                       info, level, L);
    return hipGetLastError();
  }
  const size_t smem = sizeof(T) * (size_t)4 * r * r;
  auto k = couple_factor_kernel<T>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(nparents), dim3(kCfThreads), smem, s, r, kp, Rp, segs, d_seg_start, Klu, Kpiv, Kperm,
                     Kud, W, info, level, L);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(couple_dinv_kernel<T>, dim3(nparents), dim3(kCfThreads), 0, s, 2 * r, kp, (const T*)Klu, Kinv);
  return hipGetLastError();
}
template hipError_t launch_couple_factor<double>(hipStream_t, int, int, int, int, const double*, const int32_t*,
                                                 double*, int32_t*, int32_t*, double*, double*, double*,
                                                 unsigned long long*, int, int);
template hipError_t launch_couple_factor<float>(hipStream_t, int, int, int, int, const float*, const int32_t*,
                                                float*, int32_t*, int32_t*, float*, float*, float*,
                                                unsigned long long*, int, int);

// ---------------------------------------------------------------------------
// couple_solve: one wave per parent, columns in groups of kCsCols
// ---------------------------------------------------------------------------
constexpr int kCsCols = 4;

template <typename T, int TRANS>
__global__ __launch_bounds__(64) void couple_solve_kernel(int r, int kp, int nrhs, const T* __restrict__ segs,
                                                          const int32_t* __restrict__ seg_start,
                                                          const T* __restrict__ Klu, const int32_t* __restrict__ Kperm,
                                                          const T* __restrict__ Kud, T* __restrict__ w) {
  const int g = blockIdx.x;
  const int a = 2 * g, b = 2 * g + 1;
  const int n2 = 2 * r;
  const int lane = threadIdx.x;
  const int64_t elems = (int64_t)r * nrhs;
  const T* Kf = Klu + (int64_t)g * kp * kp;
  const int32_t* pm = Kperm + (int64_t)g * kp;
  const T* kud = Kud + (int64_t)g * kp;
  T* wg = w + (int64_t)g * n2 * nrhs;
  for (int cbase = 0; cbase < nrhs; cbase += kCsCols) {
    T x[2][kCsCols];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int row = s * 64 + lane;
#pragma unroll
      for (int c = 0; c < kCsCols; ++c) {
        T v = T(0);
        if (row < n2 && cbase + c < nrhs) {
          const int src = TRANS ? row : pm[row];
          const int node = src < r ? a : b;
          v = seg_sum(segs, seg_start, node, elems, (src % r) + (int64_t)(cbase + c) * r);
        }
        x[s][c] = v;
      }
    }
    wave_lu_solve<T, kCsCols, TRANS>(x, Kf, kud, n2, kp, lane);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int row = s * 64 + lane;
#pragma unroll
      for (int c = 0; c < kCsCols; ++c)
        if (row < n2 && cbase + c < nrhs) {
          const int dst = TRANS ? pm[row] : row;
          wg[dst + (int64_t)(cbase + c) * n2] = x[s][c];
        }
    }
  }
}

// Same solve for 2r <= 64 with the factor staged in LDS, lane i owning row i
// of the right-hand sides: each substitution step reads one LDS entry per lane
// (prefetched a step ahead) and broadcasts x_j with readlane.  The loops are
// not unrolled: the code runs once per wave and would otherwise be bound by
// instruction fetch.
template <typename T, int TRANS>
__global__ __launch_bounds__(64) void couple_solve_reg_kernel(int r, int kp, int nrhs, const T* __restrict__ segs,
                                                              const int32_t* __restrict__ seg_start,
                                                              const T* __restrict__ Klu,
                                                              const int32_t* __restrict__ Kperm,
                                                              const T* __restrict__ Kud, T* __restrict__ w) {
  __shared__ T Ks[64 * 64];  // Ks[j * 64 + i] = K(i, j) (TRANS: K(j, i))
  const int g = blockIdx.x;
  const int a = 2 * g, b = 2 * g + 1;
  const int n2 = 2 * r;
  const int lane = threadIdx.x;
  const int64_t elems = (int64_t)r * nrhs;
  const T* Kf = Klu + (int64_t)g * kp * kp;
  const int32_t* pm = Kperm + (int64_t)g * kp;
  T* wg = w + (int64_t)g * n2 * nrhs;
  const bool valid = lane < n2;
  const int ln = valid ? lane : 0;
  for (int j = 0; j < n2; ++j) Ks[j * 64 + lane] = TRANS ? Kf[j + (int64_t)ln * kp] : Kf[ln + (int64_t)j * kp];
  const T dinv = valid ? Kud[(int64_t)g * kp + lane] : T(1);
  const int src = TRANS ? ln : pm[ln];
  const int64_t sbase = (int64_t)seg_start[src < r ? a : b] * elems + (src % r);
  const int dst = TRANS ? pm[ln] : ln;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int c0 = 0; c0 < nrhs; c0 += kCsCols) {
    T x[kCsCols];
#pragma unroll
    for (int c = 0; c < kCsCols; ++c) {
      const T v = segs[sbase + (int64_t)min(c0 + c, nrhs - 1) * r];
      x[c] = (valid && c0 + c < nrhs) ? v : T(0);
    }
    // forward: L (unit lower) or U^T (lower); backward: U or L^T (unit upper)
    T f = Ks[lane];
    for (int j = 0; j < n2; ++j) {
      const T fj = f;
      f = Ks[min(j + 1, 63) * 64 + lane];
      const T dj = TRANS ? bcast(dinv, j) : T(1);
#pragma unroll
      for (int c = 0; c < kCsCols; ++c) {
        const T xj = bcast(x[c], j) * dj;
        if (TRANS && lane == j) x[c] = xj;
        else if (lane > j) x[c] -= fj * xj;
      }
    }
    f = Ks[(n2 - 1) * 64 + lane];
    for (int j = n2 - 1; j >= 0; --j) {
      const T fj = f;
      f = Ks[max(j - 1, 0) * 64 + lane];
      const T dj = TRANS ? T(1) : bcast(dinv, j);
#pragma unroll
      for (int c = 0; c < kCsCols; ++c) {
        const T xj = bcast(x[c], j) * dj;
        if (!TRANS && lane == j) x[c] = xj;
        else if (lane < j) x[c] -= fj * xj;
      }
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < kCsCols; ++c)
        if (c0 + c < nrhs) wg[dst + (int64_t)(c0 + c) * n2] = x[c];
    }
  }
}

// Solves with an explicit K^{-1} (factors from couple_factor_inv_kernel or
// couple_factor_inv2_kernel): one wave per parent, lane i forms rows
// i + 64 s (s < NS) of w = K^{-1} rhs (TRANS: K^{-T} rhs), the
// right-hand-side columns broadcast from LDS.
template <typename T, int TRANS, int NS>
__global__ __launch_bounds__(64) void couple_apply_kernel(int r, int nrhs, const T* __restrict__ segs,
                                                          const int32_t* __restrict__ seg_start,
                                                          const T* __restrict__ Kinv, T* __restrict__ w) {
  __shared__ T xs[kCsCols * 64 * NS];
  const int g = blockIdx.x;
  const int a = 2 * g, b = 2 * g + 1;
  const int n2 = 2 * r;
  const int lane = threadIdx.x;
  const int64_t elems = (int64_t)r * nrhs;
  const T* Kg = Kinv + (int64_t)g * n2 * n2;
  T* wg = w + (int64_t)g * n2 * nrhs;
  bool valid[NS];
  int ln[NS];
  int64_t sbase[NS];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int row = 64 * sl + lane;
    valid[sl] = row < n2;
    ln[sl] = valid[sl] ? row : 0;
    sbase[sl] = (int64_t)seg_start[ln[sl] < r ? a : b] * elems + (ln[sl] % r);
  }
  for (int c0 = 0; c0 < nrhs; c0 += kCsCols) {
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
#pragma unroll
      for (int c = 0; c < kCsCols; ++c) {
        const T v = segs[sbase[sl] + (int64_t)min(c0 + c, nrhs - 1) * r];
        xs[c * 64 * NS + 64 * sl + lane] = (valid[sl] && c0 + c < nrhs) ? v : T(0);
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    T acc[NS][kCsCols];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
#pragma unroll
      for (int c = 0; c < kCsCols; ++c) acc[sl][c] = T(0);
#pragma unroll 8
    for (int k = 0; k < n2; ++k) {
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        const T kv = TRANS ? Kg[k + (int64_t)ln[sl] * n2] : Kg[ln[sl] + (int64_t)k * n2];
#pragma unroll
        for (int c = 0; c < kCsCols; ++c) acc[sl][c] += kv * xs[c * 64 * NS + k];
      }
    }
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
      if (valid[sl]) {
#pragma unroll
        for (int c = 0; c < kCsCols; ++c)
          if (c0 + c < nrhs) wg[64 * sl + lane + (int64_t)(c0 + c) * n2] = acc[sl][c];
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <typename T>
hipError_t launch_couple_solve(hipStream_t s, int trans, int nparents, int r, int kp, int nrhs, const T* segs,
                               const int32_t* d_seg_start, const T* Klu, const int32_t* Kperm, const T* Kud, T* w) {
  if (nparents == 0 || r == 0 || nrhs == 0) return hipSuccess;
  if (couple_uses_inverse(r)) {
#define HODLR_CA(TR, NS)                                                                                            \
  hipLaunchKernelGGL((couple_apply_kernel<T, TR, NS>), dim3(nparents), dim3(64), 0, s, r, nrhs, segs, d_seg_start, \
                     Klu, w)
    if (2 * r > 64) {
      if (trans) HODLR_CA(1, 2);
      else HODLR_CA(0, 2);
    } else {
      if (trans) HODLR_CA(1, 1);
      else HODLR_CA(0, 1);
    }
#undef HODLR_CA
    return hipGetLastError();
  }
  if (2 * r <= 64) {
    if (trans)
      hipLaunchKernelGGL((couple_solve_reg_kernel<T, 1>), dim3(nparents), dim3(64), 0, s, r, kp, nrhs, segs,
                         d_seg_start, Klu, Kperm, Kud, w);
    else
      hipLaunchKernelGGL((couple_solve_reg_kernel<T, 0>), dim3(nparents), dim3(64), 0, s, r, kp, nrhs, segs,
                         d_seg_start, Klu, Kperm, Kud, w);
    return hipGetLastError();
  }
  if (trans)
    hipLaunchKernelGGL((couple_solve_kernel<T, 1>), dim3(nparents), dim3(64), 0, s, r, kp, nrhs, segs, d_seg_start,
                       Klu, Kperm, Kud, w);
  else
    hipLaunchKernelGGL((couple_solve_kernel<T, 0>), dim3(nparents), dim3(64), 0, s, r, kp, nrhs, segs, d_seg_start,
                       Klu, Kperm, Kud, w);
  return hipGetLastError();
}
template hipError_t launch_couple_solve<double>(hipStream_t, int, int, int, int, int, const double*, const int32_t*,
                                                const double*, const int32_t*, const double*, double*);
template hipError_t launch_couple_solve<float>(hipStream_t, int, int, int, int, int, const float*, const int32_t*,
                                               const float*, const int32_t*, const float*, float*);

}  // namespace hodlr
