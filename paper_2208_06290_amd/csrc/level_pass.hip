// Fused per-level pass over row tiles (Alg. "a:gpuf" batched GEMMs and
// Alg. "a:gpus" batched GEMMs, restated on row tiles):
//
//   update : Z(tile, 0:nz) -= A1(tile, 0:ka) * W_node(0:ka, 0:nz)
//            factor: Y_big(I_a, 1:R_l) -= Y_a W_a        (eq. "e:node2")
//            solve : x(I_a) -= Y_a w_a                    (eq. "e:node4")
//   product: P_tile(0:kb, 0:nz) = B1(tile, 0:kb)^T * Z(tile, 0:nz)
//            the partial sums of V^T Y (eq. "e:node1" right side and the T
//            blocks of eq. "e:k") or of V^T x (eq. "e:node3") for the next level
//
// Workgroup = 256 threads = 4 waves; tile <= 256 rows (wave w owns rows
// 64w..64w+63), one chunk of 64 columns of Z and one chunk of <= 64 columns
// of B1; the four waves' partial products are summed in LDS in a fixed order.
//
// Two kernels: level_pass_fast_kernel when tile heights, ka and kb are
// multiples of 16 (the common case), level_pass_kernel otherwise.
#include "mfma.h"

#include <algorithm>
#include <type_traits>

namespace hodlr {

constexpr int kLpThreads = 256;

// General kernel: any tile height and any sizes, with clamped loads and
// masked values and stores.  The updated Z tile stays in the accumulator
// registers and feeds the product directly as B operand: in the accumulator
// layout each 4-register group holds 4 rows x 16 columns, one K-step.
template <typename TZ, typename SA, typename SB, int MB>
__global__ __launch_bounds__(kLpThreads, 2) void level_pass_kernel(const Tile* __restrict__ tiles, int zchunks,
                                                                   int bchunks, TZ* Z, int64_t ldz, int nz,
                                                                   const SA* __restrict__ A1, int64_t lda, int ka,
                                                                   const TZ* __restrict__ W, int64_t w_ld,
                                                                   int64_t w_pstride, int node_shift,
                                                                   const SB* __restrict__ B1, int64_t ldb,
                                                                   int kb_total, TZ* __restrict__ P, GroupStrides gs) {
  using M = Mfma<TZ>;
  using V = typename M::V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TZ* Ws = reinterpret_cast<TZ*>(smem_raw);   // update phase: W chunk [k][64]
  TZ* red = reinterpret_cast<TZ*>(smem_raw);  // product phase: [4 waves][MB*16][64]

  const int lid = (int)xcd_remap(blockIdx.x, gridDim.x);  // grid < 2^31: 32-bit index math
  const int bchunk = lid % bchunks;
  const int zchunk = (lid / bchunks) % zchunks;
  const int tile = lid / (bchunks * zchunks);
  const Tile tl = tiles[tile];
  const int nrows = tl.nrows;
  // first row of the tile in each operand (rows inside a tile are contiguous)
  TZ* Zt = Z + group_row(tl.row0, gs.z);
  const SA* At = A1 ? A1 + group_row(tl.row0, gs.a) : A1;
  const SB* Bt = B1 ? B1 + group_row(tl.row0, gs.b) : B1;
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

  // loads are clamped into range and masked with a select: no branches, nothing drains the queue
  auto load_z = [&](int rb, V (&dst)[4]) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = wr0 + 16 * rb + M::crow(lq, t);
        const int col = c0 + 16 * cb + li;
        const bool ok = row < nrows && col < nz;
        const TZ v = Zt[min(row, nrows - 1) + (int64_t)min(col, nz - 1) * ldz];
        dst[cb][t] = ok ? v : TZ(0);
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
      const int rowc = min(row, nrows - 1);
      for (int ks = 0; ks < nks; ++ks) {
        const int kk = 4 * ks + lq;
        const TZ av = -(TZ)At[rowc + (int64_t)min(kk, ka - 1) * lda];
        const TZ a = (row < nrows && kk < ka) ? av : TZ(0);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          acc[cb] = M::mma(a, Ws[kk * 64 + 16 * cb + li], acc[cb]);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int rr = wr0 + 16 * rb + M::crow(lq, t);
          const int col = c0 + 16 * cb + li;
          if (cb < ncb && rr < nrows && col < nz) Zt[rr + (int64_t)col * ldz] = acc[cb][t];
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
          const TZ bv = (TZ)Bt[min(rr, nrows - 1) + (int64_t)(kc0 + min(kr, kb - 1)) * ldb];
          bo[mb] = (rr < nrows && kr < kb) ? bv : TZ(0);
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            pacc[mb][cb] = M::mma(bo[mb], acc[cb][t], pacc[mb][cb]);
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
    TZ* Pt = P + (int64_t)tile * kb_total * nz;
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


// Fast kernel: tile heights, ka and kb are multiples of 16 (nz is free).  The
// update is computed transposed, Z^T -= W^T A1^T, so that the 16 lanes of a
// row group hold 16 consecutive rows of one column of Z: every load and store
// of Z and A1 covers whole 128-byte lines, addressed as a lane-uniform base
// plus one 32-bit lane offset (buffer addressing).  For the product the
// updated block is turned around through a per-wave LDS buffer (the
// contraction runs over rows, which MFMA takes on its 4-deep K side); B1 is
// loaded coalesced and turned around the same way.  A chunk is 16 NCB
// columns of Z (NCB = 1 for narrow right-hand sides, else 4).  Columns past
// nz are computed on zeros and never stored; their loads are redirected to an
// in-range column, so no access leaves the operands.  RP = 2 (4-byte Z, tile
// heights multiples of 32): each lane holds two consecutive rows, loaded and
// stored as one 8-byte access, so 16 lanes still cover a whole 128-byte line;
// the even and the odd rows form two 16-row MFMA blocks (the product's sum
// over rows does not depend on their order).
constexpr int kZtLd = 17;  // padded row length of the per-wave 16 x 16 turn-around buffer

template <typename TZ, typename SA, typename SB, int MB, int NKS, int NCB, int MODE, int RP, bool BF, bool BLK>
__global__ __launch_bounds__(kLpThreads, (MB > 2 || NKS > 8) ? 2 : 3) void level_pass_fast_kernel(
    const Tile* __restrict__ tiles, int zchunks, int c_base, int bchunks, TZ* Z, int64_t ldz, int nz, const SA* __restrict__ A1,
    int64_t lda, const TZ* __restrict__ W, int64_t w_ld, int64_t w_pstride, int node_shift,
    const SB* __restrict__ B1, int64_t ldb, int kb_total, TZ* __restrict__ P, GroupStrides gs) {
  using M = Mfma<TZ>;
  using V = typename M::V;
  constexpr int ka = 4 * NKS;
  constexpr int kb = 16 * MB;  // B1 columns of this chunk (kb_total is a multiple of 16)
  constexpr int kCw = 16 * NCB;  // Z columns of a chunk
  constexpr int kBtLd = 16 * MB + 1;
  constexpr int kWave = 16 * kZtLd + 16 * kBtLd;
  constexpr bool prod = MB > 0;
  static_assert(MODE != 2 || NCB == 1, "a chunk with a ragged column count is one 16-column block");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TZ* Ws = reinterpret_cast<TZ*>(smem_raw);   // W chunk [ka][kCw]
  TZ* red = reinterpret_cast<TZ*>(smem_raw);  // end of the product: [2][kb][kCw]

  const int lid = (int)xcd_remap(blockIdx.x, gridDim.x);  // grid < 2^31: 32-bit index math
  const int bchunk = lid % bchunks;
  const int zchunk = (lid / bchunks) % zchunks;
  const int tile = lid / (bchunks * zchunks);
  const Tile tl = tiles[tile];
  const int nrows = tl.nrows;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lq = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: addresses stay scalar
  const int c0 = c_base + zchunk * kCw;
  const int ncz = MODE == 0 ? kCw : min(kCw, nz - c0);  // valid columns of this chunk
  const int wr0 = 64 * w;
  const int nrb = max(0, min(4 / RP, (nrows - wr0) >> (RP == 2 ? 5 : 4)));  // 16 RP-row blocks of this wave
  const int kc0 = bchunk * 64;
  TZ* zt = Ws + kCw * ka + w * kWave;
  TZ* bt = zt + 16 * kZtLd;

  if (NKS > 0) {
    const int nd = tl.node >> node_shift;
    const TZ* Wn = W + (int64_t)(nd >> 1) * w_pstride + (int64_t)(nd & 1) * ka;
    if constexpr (BF) {
      // W converted to bfloat16 once, as the update's A operands: element
      // (k, c) to group k / 16, block c / 16, lane (k % 4, c % 16), slot
      // (k / 4) % 4, so that one 8-byte read gives a lane its four values
      __bf16* Wb = reinterpret_cast<__bf16*>(Ws);
      for (int e = tid; e < kCw * ka; e += kLpThreads) {
        const int c = e % kCw, k = e / kCw;
        const TZ v = (c < ncz) ? Wn[k + (int64_t)(c0 + c) * w_ld] : TZ(0);
        Wb[((((k >> 4) * NCB + (c >> 4)) * 4 + (k & 3)) * 16 + (c & 15)) * 4 + ((k >> 2) & 3)] = (__bf16)v;
      }
    } else {
      for (int e = tid; e < kCw * ka; e += kLpThreads) {
        const int c = e % kCw, k = e / kCw;
        Ws[e] = (c < ncz) ? Wn[k + (int64_t)(c0 + c) * w_ld] : TZ(0);
      }
    }
  }

  // first row of this wave in each operand (rows inside a tile are contiguous).
  // BLK (product-only passes whose 64-column chunk would need byte offsets
  // past 2^31, e.g. the FP64 matvec projections at N = 2^22) takes a buffer
  // resource per 16-column block of Z and of B1, so offsets stay below 16
  // columns of the leading dimension; otherwise one resource per operand.
  static_assert(!BLK || NKS == 0, "per-block resources only in product-only passes");
  constexpr bool kBlk = BLK;
  constexpr int kZr = kBlk ? NCB : 1;
  constexpr int kBr = kBlk && MB > 0 ? MB : 1;
  __amdgpu_buffer_rsrc_t zr[kZr];
#pragma unroll
  for (int cb = 0; cb < kZr; ++cb) {
    // MODE 1: blocks past the valid columns re-read the last valid one
    const int blk = !kBlk ? 0 : MODE == 1 ? min(cb, (ncz >> 4) - 1) : cb;
    zr[cb] = buf_rsrc(Z + group_row(tl.row0, gs.z) + wr0 + (int64_t)(c0 + 16 * blk) * ldz);
  }
  const auto ar = buf_rsrc(NKS > 0 ? A1 + group_row(tl.row0, gs.a) + wr0 : A1);  // A1 / B1 are null when unused
  __amdgpu_buffer_rsrc_t br[kBr];
#pragma unroll
  for (int q = 0; q < kBr; ++q)
    br[q] = buf_rsrc(prod ? B1 + group_row(tl.row0, gs.b) + wr0 + (int64_t)(kc0 + 16 * q) * ldb : B1);
  const uint32_t zrow = (uint32_t)(RP * li) * (uint32_t)sizeof(TZ);
  const uint32_t zl = zrow + (uint32_t)((int64_t)M::crow_l(lq) * ldz) * (uint32_t)sizeof(TZ);
  const uint32_t al = (uint32_t)(RP * li + (int64_t)lq * lda) * (uint32_t)sizeof(SA);
  const uint32_t bl = (uint32_t)(RP * li + (int64_t)lq * ldb) * (uint32_t)sizeof(SB);
  constexpr uint32_t kRbRows = 16 * RP;  // rows of one row block
  // Z(16 rb + li, c0 + 16 cb + crow(lq, t)) is register t of the Z^T accumulator
  // block cb (RP = 2: rows 32 rb + 2 li + h of block h).  The lane-uniform
  // column part is clamped into the chunk; a lane whose own column is past nz
  // drops its lane part and reads the clamped column instead (its value is
  // replaced by zero).
  // MODE 0: every column of the chunk is valid; MODE 1: the valid columns
  // are whole 16-column blocks (later blocks re-read the last valid one, a
  // lane-uniform clamp); MODE 2: any count (per-lane test)
  auto zok = [&](int cb, int t) -> bool {
    if (MODE == 0) return true;
    if (MODE == 1) return 16 * cb < ncz;
    return 16 * cb + M::crow_u(t) + M::crow_l(lq) < ncz;
  };
  // the resource of block cb and the column offset inside it
  auto zrs = [&](int cb) { return zr[kBlk ? cb : 0]; };
  auto zso = [&](int cb, int t) -> uint32_t {
    const int col = MODE == 0   ? 16 * cb + M::crow_u(t)
                    : MODE == 1 ? 16 * min(cb, (ncz >> 4) - 1) + M::crow_u(t)
                                : min(16 * cb + M::crow_u(t), ncz - 1);
    const int base = !kBlk ? 0 : MODE == 1 ? 16 * min(cb, (ncz >> 4) - 1) : 16 * cb;
    return (uint32_t)((int64_t)(col - base) * ldz * (int64_t)sizeof(TZ));
  };
  auto zvo = [&](int rb, int cb, int t) -> uint32_t {
    return (MODE < 2 || zok(cb, t) ? zl : zrow) + kRbRows * (uint32_t)rb * (uint32_t)sizeof(TZ);
  };
  auto load_z = [&](int rb, V (&d0)[NCB], V (&d1)[NCB]) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        TZ v0, v1 = TZ(0);
        if (RP == 2) Buf2<TZ>::load(zrs(cb), zvo(rb, cb, t), zso(cb, t), v0, v1);
        else v0 = Buf<TZ>::load(zrs(cb), zvo(rb, cb, t), zso(cb, t));
        d0[cb][t] = zok(cb, t) ? v0 : TZ(0);
        d1[cb][t] = zok(cb, t) ? v1 : TZ(0);
      }
  };
  // B operand of the update: -A1(row, 4 ks + lq) for the lane's row(s)
  auto load_a = [&](int rb, TZ (&d0)[NKS > 0 ? NKS : 1], TZ (&d1)[NKS > 0 ? NKS : 1]) {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const uint32_t vo = al + kRbRows * (uint32_t)rb * (uint32_t)sizeof(SA);
      const uint32_t so = (uint32_t)((int64_t)(4 * ks) * lda * (int64_t)sizeof(SA));
      SA x0, x1 = SA(0);
      if (RP == 2) Buf2<SA>::load(ar, vo, so, x0, x1);
      else x0 = Buf<SA>::load(ar, vo, so);
      d0[ks] = -(TZ)x0;
      d1[ks] = -(TZ)x1;
    }
  };
  // B1(row, kc0 + 4 i + lq); the last B1 chunk may hold fewer than kb
  // columns (a multiple of 16): the others read column kc0 and are zeroed
  const int kbc = prod ? min(kb, kb_total - kc0) : 0;
  auto load_b = [&](int rb, TZ (&d0)[MB > 0 ? 4 * MB : 1], TZ (&d1)[MB > 0 ? 4 * MB : 1]) {
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) {
      const bool ok = 4 * i < kbc;  // uniform
      const uint32_t vo = bl + kRbRows * (uint32_t)rb * (uint32_t)sizeof(SB);
      // column 4 i (inside block i / 4 of its own resource when kBlk), or
      // column kc0 when past the valid ones
      const int col = ok ? (kBlk ? 4 * (i % 4) : 4 * i) : 0;
      const uint32_t so = (uint32_t)((int64_t)col * ldb * (int64_t)sizeof(SB));
      const auto rs = kBlk && ok ? br[kBlk ? i / 4 : 0] : br[0];
      SB x0, x1 = SB(0);
      if (RP == 2) Buf2<SB>::load(rs, vo, so, x0, x1);
      else x0 = Buf<SB>::load(rs, vo, so);
      d0[i] = ok ? (TZ)x0 : TZ(0);
      d1[i] = ok ? (TZ)x1 : TZ(0);
    }
  };

  V pacc[MB > 0 ? MB : 1][NCB];
#pragma unroll
  for (int mb = 0; mb < (MB > 0 ? MB : 1); ++mb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) pacc[mb][cb] = vzero<V>();

  // update of one 16-row MFMA block, and its contribution to the product
  auto update = [&](V (&acc)[NCB], const TZ (&acur)[NKS > 0 ? NKS : 1]) {
    if constexpr (BF) {
      // groups of four K-steps as one bfloat16 MFMA (NKS is a multiple of 4);
      // the row's A values are packed once per group, W was packed when staged
      const s4* Wp = reinterpret_cast<const s4*>(Ws);
#pragma unroll
      for (int g = 0; g < NKS / 4; ++g) {
        TZ av4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) av4[j] = acur[4 * g + j];
        const s4 ap = pack_bf16(av4);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = mma_bf16(Wp[((g * NCB + cb) * 4 + lq) * 16 + li], ap, acc[cb]);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[cb] = M::mma(Ws[(4 * ks + lq) * kCw + 16 * cb + li], acur[ks], acc[cb]);
    }
  };
  auto stage_b = [&](const TZ (&bcur)[MB > 0 ? 4 * MB : 1]) {
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) bt[li * kBtLd + 4 * i + lq] = bcur[i];
  };
  auto product = [&](const V (&acc)[NCB]) {
    // P(j, c) += sum_r B1(r, j) Z(r, c); K-step kk takes rows 4 kk + lq; the
    // turned-around B1 block is read into registers once
    TZ bv[4][MB > 0 ? MB : 1];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) bv[kk][mb] = bt[(4 * kk + lq) * kBtLd + 16 * mb + li];
    // bfloat16: the B1 operands packed once for every Z block
    s4 bp[BF && MB > 0 ? MB : 1];
    if constexpr (BF) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        TZ b4v[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) b4v[kk] = bv[kk][mb];
        bp[mb] = pack_bf16(b4v);
      }
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int t = 0; t < 4; ++t) zt[li * kZtLd + M::crow(lq, t)] = acc[cb][t];
      if constexpr (BF) {
        TZ zv4[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) zv4[kk] = zt[(4 * kk + lq) * kZtLd + li];
        const s4 zp = pack_bf16(zv4);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) pacc[mb][cb] = mma_bf16(bp[mb], zp, pacc[mb][cb]);
      } else {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const TZ zv = zt[(4 * kk + lq) * kZtLd + li];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) pacc[mb][cb] = M::mma(bv[kk][mb], zv, pacc[mb][cb]);
        }
      }
    }
  };

  if (NKS > 0) __syncthreads();  // W chunk staged
  // no software prefetch: latency is hidden by the other resident waves
#pragma unroll 1
  for (int rb = 0; rb < nrb; ++rb) {
    V acc0[NCB], acc1[NCB];
    TZ a0[NKS > 0 ? NKS : 1], a1[NKS > 0 ? NKS : 1];
    TZ b0[MB > 0 ? 4 * MB : 1], b1[MB > 0 ? 4 * MB : 1];
    load_z(rb, acc0, acc1);
    if (NKS > 0) load_a(rb, a0, a1);
    if (prod) {
      load_b(rb, b0, b1);
      stage_b(b0);
    }
    if (NKS > 0) {
      update(acc0, a0);
      if (RP == 2) update(acc1, a1);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (zok(cb, t)) {
            if (RP == 2) Buf2<TZ>::store(acc0[cb][t], acc1[cb][t], zrs(cb), zvo(rb, cb, t), zso(cb, t));
            else Buf<TZ>::store(acc0[cb][t], zrs(cb), zvo(rb, cb, t), zso(cb, t));
          }
    }
    if (prod) {
      product(acc0);
      if (RP == 2) {
        stage_b(b1);  // after the even block's reads of bt (in order within the wave)
        product(acc1);
      }
    }
  }

  if (prod) {
    // partial products of the four waves, summed in the fixed order (w0 + w2) + (w1 + w3)
    // through a two-slot LDS buffer that reuses the W chunk and turn-around space
    __syncthreads();
    if (w < 2) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int t = 0; t < 4; ++t)
            red[(w * kb + 16 * mb + M::crow(lq, t)) * kCw + 16 * cb + li] = pacc[mb][cb][t];
    }
    __syncthreads();
    if (w >= 2) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            TZ* r = red + ((w - 2) * kb + 16 * mb + M::crow(lq, t)) * kCw + 16 * cb + li;
            *r = *r + pacc[mb][cb][t];
          }
    }
    __syncthreads();
    TZ* Pt = P + (int64_t)tile * kb_total * nz;
    for (int e = tid; e < kb * kCw; e += kLpThreads) {
      const int kr = e % kb, cw = e / kb;
      if (cw < ncz && kr < kbc)
        Pt[(kc0 + kr) + (int64_t)(c0 + cw) * kb_total] = red[kr * kCw + cw] + red[(kb + kr) * kCw + cw];
    }
  }
}

template <typename TZ, typename SA, typename SB, int MB, int NKS, int NCB, int MODE, int RP, bool BF, bool BLK>
static hipError_t launch_part(hipStream_t s, int ntiles, int zchunks, int c_base, int nz, int bchunks,
                              const Tile* tiles, TZ* Z, int64_t ldz, const SA* A1, int64_t lda, const TZ* W,
                              int64_t w_ld, int64_t w_pstride, int node_shift, const SB* B1, int64_t ldb, int kb, TZ* P,
                              GroupStrides gs) {
  if (zchunks == 0) return hipSuccess;
  constexpr int kCw = 16 * NCB;
  const size_t smem_main = sizeof(TZ) * (kCw * 4 * (size_t)NKS + 4 * (16 * kZtLd + 16 * (16 * MB + 1)));
  const size_t smem_red = MB > 0 ? sizeof(TZ) * 2 * 16 * MB * kCw : 0;
  const size_t smem = smem_main > smem_red ? smem_main : smem_red;
  const int64_t grid = (int64_t)ntiles * zchunks * bchunks;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  auto k = level_pass_fast_kernel<TZ, SA, SB, MB, NKS, NCB, MODE, RP, BF, BLK>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kLpThreads), smem, s, tiles, zchunks, c_base, bchunks, Z, ldz, nz,
                     A1, lda, W, w_ld, w_pstride, node_shift, B1, ldb, kb, P, gs);
  return hipGetLastError();
}

// Columns of Z in up to three launches: chunks of 64, then the whole 16-column
// blocks that are left as one narrower chunk, then a last partial block
// (per-lane column test).  Every launch computes only columns that exist.
template <typename TZ, typename SA, typename SB, int MB, int NKS, int RP, bool BF, bool BLK>
static hipError_t launch_fast(hipStream_t s, int ntiles, int nz, int bchunks, const Tile* tiles, TZ* Z, int64_t ldz,
                              const SA* A1, int64_t lda, const TZ* W, int64_t w_ld, int64_t w_pstride,
                              int node_shift, const SB* B1, int64_t ldb, int kb, TZ* P, GroupStrides gs) {
  const int n64 = nz / 64, nb = (nz % 64) / 16, tail = nz % 16;
  hipError_t e = launch_part<TZ, SA, SB, MB, NKS, 4, 0, RP, BF, BLK>(s, ntiles, n64, 0, nz, bchunks, tiles, Z, ldz, A1, lda, W,
                                                         w_ld, w_pstride, node_shift, B1, ldb, kb, P, gs);
  if (e != hipSuccess) return e;
  const int cb = 64 * n64;
#define HODLR_LPB(NCBV)                                                                                          \
  e = launch_part<TZ, SA, SB, MB, NKS, NCBV, 0, RP, BF, BLK>(s, ntiles, 1, cb, nz, bchunks, tiles, Z, ldz, A1, lda, W, w_ld,  \
                                                 w_pstride, node_shift, B1, ldb, kb, P, gs)
  if (nb == 1) HODLR_LPB(1);
  else if (nb == 2) HODLR_LPB(2);
  else if (nb == 3) HODLR_LPB(3);
#undef HODLR_LPB
  if (e != hipSuccess) return e;
  return launch_part<TZ, SA, SB, MB, NKS, 1, 2, RP, BF, BLK>(s, ntiles, tail ? 1 : 0, cb + 16 * nb, nz, bchunks, tiles, Z, ldz, A1,
                                                lda, W, w_ld, w_pstride, node_shift, B1, ldb, kb, P, gs);
}

template <typename TZ, typename SA, typename SB, int MB, int RP, bool BF, bool BLK>
static hipError_t launch_fast_nks(int nks, hipStream_t s, int ntiles, int nz, int bchunks, const Tile* tiles, TZ* Z,
                                  int64_t ldz, const SA* A1, int64_t lda, const TZ* W, int64_t w_ld,
                                  int64_t w_pstride, int node_shift, const SB* B1, int64_t ldb, int kb, TZ* P,
                                  GroupStrides gs) {
#define HODLR_LPF(NKSV)                                                                                       \
  return launch_fast<TZ, SA, SB, MB, NKSV, RP, BF, BLK>(s, ntiles, nz, bchunks, tiles, Z, ldz, A1, lda, W, w_ld, w_pstride,      \
                                                 node_shift, B1, ldb, kb, P, gs)
  if constexpr (BLK) {  // product-only
    if (nks != 0) return hipErrorInvalidValue;
    HODLR_LPF(0);
  } else {
  switch (nks) {
    case 0: HODLR_LPF(0);
    case 4: HODLR_LPF(4);
    case 8: HODLR_LPF(8);
    case 12: HODLR_LPF(12);
    default: HODLR_LPF(16);
  }
  }
#undef HODLR_LPF
}

template <typename TZ, typename SA, typename SB, int RP, bool BF, bool BLK = false>
static hipError_t launch_fast_all(hipStream_t s, int ntiles, const Tile* tiles, TZ* Z, int64_t ldz, int nz,
                                  const SA* A1, int64_t lda, int ka, const TZ* W, int64_t w_ld, int64_t w_pstride,
                                  int node_shift, const SB* B1, int64_t ldb, int kb, TZ* P, GroupStrides gs) {
  const int bchunks = kb > 0 ? (kb + 63) / 64 : 1;
  const int nks = ka / 4;
#define HODLR_LPM(MBV)                                                                                            \
  return launch_fast_nks<TZ, SA, SB, MBV, RP, BF, BLK>(nks, s, ntiles, nz, bchunks, tiles, Z, ldz, A1, lda, W, w_ld,           \
                                                w_pstride, node_shift, B1, ldb, kb, P, gs)
  switch (kb > 0 ? std::min(kb, 64) / 16 : 0) {
    case 0: HODLR_LPM(0);
    case 1: HODLR_LPM(1);
    case 2: HODLR_LPM(2);
    case 3: HODLR_LPM(3);
    default: HODLR_LPM(4);
  }
#undef HODLR_LPM
}

template <typename TZ, typename SA, typename SB>
hipError_t launch_level_pass(hipStream_t s, int ntiles, const Tile* tiles, int tiles_aligned, TZ* Z, int64_t ldz,
                             int nz, const SA* A1, int64_t lda, int ka, const TZ* W, int64_t w_ld,
                             int64_t w_pstride, int node_shift, const SB* B1, int64_t ldb, int kb, TZ* P,
                             GroupStrides gs, int bf) {
  if (ntiles == 0 || nz == 0 || (ka == 0 && kb == 0)) return hipSuccess;
  const int zchunks = (nz + 63) / 64;
  const int bchunks = kb > 0 ? (kb + 63) / 64 : 1;
  if (ka > 0 && bchunks > 1) return hipErrorInvalidValue;  // an update must run once per element
  if (ka > 64) return hipErrorInvalidValue;
  const int64_t grid = (int64_t)ntiles * zchunks * bchunks;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  // byte offsets inside a 64-column chunk must stay below 2^31 for the buffer
  // addressing; product-only passes may instead address 16-column blocks
  const bool small_ld = 64 * ldz * (int64_t)sizeof(TZ) < (1ll << 31) && 64 * lda * (int64_t)sizeof(SA) < (1ll << 31) &&
                        64 * ldb * (int64_t)sizeof(SB) < (1ll << 31);
  const bool block_ld = ka == 0 && 16 * ldz * (int64_t)sizeof(TZ) < (1ll << 31) &&
                        16 * ldb * (int64_t)sizeof(SB) < (1ll << 31);
  if ((tiles_aligned & 1) && !small_ld && block_ld && kb % 16 == 0)
    return launch_fast_all<TZ, SA, SB, 1, false, true>(s, ntiles, tiles, Z, ldz, nz, A1, lda, ka, W, w_ld, w_pstride,
                                                       node_shift, B1, ldb, kb, P, gs);
  if ((tiles_aligned & 1) && small_ld && ka % 16 == 0 && kb % 16 == 0) {
    if constexpr (sizeof(TZ) == 4) {
      // 4-byte elements, tile heights multiples of 32, even leading dimensions and
      // 16-byte aligned operands (every paired access is naturally aligned): two rows per lane
      auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
      const bool pair_ok = ldz % 2 == 0 && (ka == 0 || lda % 2 == 0) && (kb == 0 || ldb % 2 == 0) && al16(Z) &&
                           (ka == 0 || al16(A1)) && (kb == 0 || al16(B1));
      // bfloat16 products only where the factorization uses them (Z and A1 both Y)
      constexpr bool kBf = std::is_same<SA, TZ>::value;
      if ((tiles_aligned & 2) && pair_ok) {
        if (kBf && bf)
          return launch_fast_all<TZ, SA, SB, 2, true>(s, ntiles, tiles, Z, ldz, nz, A1, lda, ka, W, w_ld, w_pstride,
                                                      node_shift, B1, ldb, kb, P, gs);
        return launch_fast_all<TZ, SA, SB, 2, false>(s, ntiles, tiles, Z, ldz, nz, A1, lda, ka, W, w_ld, w_pstride,
                                                     node_shift, B1, ldb, kb, P, gs);
      }
      if (kBf && bf)
        return launch_fast_all<TZ, SA, SB, 1, true>(s, ntiles, tiles, Z, ldz, nz, A1, lda, ka, W, w_ld, w_pstride,
                                                    node_shift, B1, ldb, kb, P, gs);
    }
    return launch_fast_all<TZ, SA, SB, 1, false>(s, ntiles, tiles, Z, ldz, nz, A1, lda, ka, W, w_ld, w_pstride,
                                                 node_shift, B1, ldb, kb, P, gs);
  }
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
                       A1, lda, ka, W, w_ld, w_pstride, node_shift, B1, ldb, kb, P, gs);                                \
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
  template hipError_t launch_level_pass<TZ, SA, SB>(hipStream_t, int, const Tile*, int, TZ*, int64_t, int, const SA*, \
                                                    int64_t, int, const TZ*, int64_t, int64_t, int,           \
                                                    const SB*, int64_t, int, TZ*, GroupStrides, int);
HODLR_LP_INST(double, double, double)
HODLR_LP_INST(float, float, double)
HODLR_LP_INST(float, double, float)
HODLR_LP_INST(float, float, float)
HODLR_LP_INST(double, double, float)
#undef HODLR_LP_INST

}  // namespace hodlr
