// Internal declarations of the HODLR library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hodlr.h"

namespace hodlr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Rows of one tile of a level pass: a run of <= kTileRows consecutive rows
// that lies inside one node of the pass's level.
constexpr int kTileRows = 256;
struct Tile {
  int64_t row0;
  int32_t nrows;
  int32_t node;  // node index (0-based, left to right) at the pass's level
};

// Segment of tiles summed by the reduction kernel.
constexpr int kSegTiles = 16;

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T ld_as(const void* p, int64_t i);
template <>
__device__ __forceinline__ double ld_as<double>(const void* p, int64_t i) {
  return static_cast<const double*>(p)[i];
}
template <>
__device__ __forceinline__ float ld_as<float>(const void* p, int64_t i) {
  return static_cast<const float*>(p)[i];
}

// XCD-aware block index remap: hardware hands consecutive workgroup ids to
// the 8 XCDs round robin; this maps them so that consecutive *logical* ids
// land on the same XCD (and share its L2).  Bijective for any grid size.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  constexpr int kX = 8;
  int64_t per = nblocks / kX;           // full rounds
  int64_t rem = nblocks % kX;
  int64_t x = bid % kX, j = bid / kX;
  if (j < per) {
    // xcd x owns logical ids [x*per + min(x, rem) ... ) of length per + (x < rem)
    return x * per + (x < rem ? x : rem) + j;
  }
  // tail round (only xcds x < rem have a block here)
  return x * per + x + per;
}

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).  T = compute type (double/float),
// S = storage type of the caller's D/U/V.
// ---------------------------------------------------------------------------

// leaf LU with partial pivoting; LU blocks col-major ldl x ldl per leaf (ldl % 16 == 0, lul = ldl),
// or in place (inplace = 1): leaf a's factor in rows [off_a, off_a + m_a) of lu with ld lul
// (every m_a % 16 == 0; lu may be D itself);
// invl: the inverted 16 x 16 diagonal blocks of L and U (2 x ldl/16 x 256 per leaf).
// bf = 1 (T = float): the trailing updates of the left-looking sweep take
// bfloat16 operands with FP32 accumulation; pivot search and panel stay FP32.
template <typename T, typename S>
hipError_t launch_leaf_lu(hipStream_t s, int nleaf, int ldl, const int64_t* d_leaf_off, const S* D, int64_t ldd,
                          T* lu, int64_t lul, int inplace, int32_t* piv, int32_t* perm, T* udinv, T* invl,
                          unsigned long long* info, int bf = 0);

// Leaf triangular solves on column chunks.
// trans = 0: X(I_a, :) = U_a^{-1} L_a^{-1} P_a^T B(I_a, :)
// trans = 1: X(I_a, :) = P_a L_a^{-T} U_a^{-T} B(I_a, :)
// B and X may alias (same type).
// dinv: per block 2 x (ldl/16) inverted 16 x 16 diagonal blocks ([0]: L, [1]: U) from the factorization.
// lu, lul, inplace: the leaf factors in either layout of launch_leaf_lu.
// bf = 1 (T = float, trans = 0): the block products take bfloat16 operands with
// FP32 accumulation (the leaf solve of a BF16 factorization).
template <typename T, typename S>
hipError_t launch_leaf_trsm(hipStream_t s, int trans, int nleaf, int ldl, const int64_t* d_leaf_off, const T* lu,
                            int64_t lul, int inplace, const int32_t* perm, const T* dinv, const S* B, int64_t ldb,
                            T* X, int64_t ldx, int ncols, int64_t gsb = 256, int64_t gsx = 256, int bf = 0);

// The same solves for nblk equal blocks of m rows (m <= ldl): block g's rows start at X + g * ostride.
template <typename T>
hipError_t launch_block_trsm(hipStream_t s, int trans, int nblk, int ldl, int m, int64_t ostride, const T* lu,
                             const int32_t* perm, const T* dinv, T* X, int64_t ldx, int ncols);

// Fused level pass on tiles:
//   update : Z(tile, 0:nz) -= A1(tile, 0:ka) * W_node(0:ka, 0:nz)      (if ka > 0)
//   product: P_tile(0:kb, 0:nz) = B1(tile, 0:kb)^T * Z(tile, 0:nz)      (if kb > 0)
// nd = tile.node >> node_shift; W for node nd starts at W + (nd >> 1) * w_pstride + (nd & 1) * ka, ld = w_ld.
// P_tile starts at P + tile * kb * nz, col-major ld = kb.
// tiles_aligned: bit 0 - every tile height is a multiple of 16 (enables the fast kernel);
// bit 1 - a multiple of 32 (4-byte Z: two rows per lane).
// Row addressing of the Z, A1 and B1 operands: row i of an operand lives at
// (i >> 8) * gs + (i & 255) (plus column * ld).  gs = 256 is the plain
// column-major layout; gs = 256 * ncols with ld = 256 is the row-group blocked
// layout (each 256-row group of all columns contiguous), valid when no tile
// crosses a 256-row boundary.
// bf = 1 (4-byte TZ): the products of the fast kernel take bfloat16 operands
// with FP32 accumulation (the coupling GEMMs of a BF16 factorization); tiles
// that need the general kernel are computed in FP32.
struct GroupStrides {
  int64_t z = 256, a = 256, b = 256;
};
__host__ __device__ __forceinline__ int64_t group_row(int64_t row, int64_t gs) { return (row >> 8) * gs + (row & 255); }

template <typename TZ, typename SA, typename SB>
hipError_t launch_level_pass(hipStream_t s, int ntiles, const Tile* tiles, int tiles_aligned, TZ* Z, int64_t ldz, int nz,
                             const SA* A1, int64_t lda, int ka, const TZ* W, int64_t w_ld,
                             int64_t w_pstride, int node_shift, const SB* B1, int64_t ldb, int kb, TZ* P,
                             GroupStrides gs = GroupStrides(), int bf = 0);

// Segment sums of tile partials: out[s] = sum of tiles [desc[s].x, desc[s].x + desc[s].y),
// maxy = max over s of desc[s].y (<= kSegTiles).
template <typename T>
hipError_t launch_segment_reduce(hipStream_t s, int nsegs, const int2* d_desc, int64_t elems, const T* P, T* out,
                                 int maxy);

// Coupling systems with 2r <= 128 and 2r % 16 == 0 are inverted explicitly
// (Gauss-Jordan with partial pivoting; four waves up to 2r = 64, eight
// beyond, two rows a lane): the factor stores K^{-1} (2r x 2r,
// col-major) in place of the LU, W receives K^{-1} rhs directly and the solves
// apply K^{-1} or its transpose.  Other ranks keep the LU, its 16 x 16 diagonal
// inverses and the block solver.
__host__ __device__ inline bool couple_uses_inverse(int r) { return r > 0 && 2 * r <= 128 && (2 * r) % 16 == 0; }

// Coupling factor for all parents of one level (children have rank r, W has Rp columns);
// K factors stored kp x kp (kp = 2r rounded up to 16); W gets the unsolved right-hand
// sides (LU) or the solved ones (explicit inverse).
// Segments of child node c: [seg_start[c], seg_start[c+1]), each r x (Rp + r) col-major.
template <typename T>
hipError_t launch_couple_factor(hipStream_t s, int nparents, int r, int kp, int Rp, const T* segs,
                                const int32_t* d_seg_start, T* Klu, int32_t* Kpiv, int32_t* Kperm, T* Kud, T* Kinv,
                                T* W, unsigned long long* info, int level, int L);

// Coupling solve for all parents of one level: w = K^{-1} rhs (trans=0) or K^{-T} rhs.
// rhs rows of child c come from its segments (r x nrhs each); w is 2r x nrhs per parent.
template <typename T>
hipError_t launch_couple_solve(hipStream_t s, int trans, int nparents, int r, int kp, int nrhs, const T* segs,
                               const int32_t* d_seg_start, const T* Klu, const int32_t* Kperm, const T* Kud, T* w);

// Pairwise tree sum out[i] = in[2i] + in[2i+1] (blocks of elems doubles).
hipError_t launch_tree_sum(hipStream_t s, int nnodes, int64_t elems, const double* in, double* out);

// Projection tree: for l = 1..L, the 2^l node sums (R x nrhs each, col-major ld R) of level l
// start at node slot (2^l - 2); slot k begins at tree + k * R * nrhs.
__host__ __device__ inline int64_t tree_slot(int l, int node) { return ((int64_t)1 << l) - 2 + node; }

// y = op(D) x + U G per leaf (FP64 arithmetic) from the projection tree.
template <typename S>
hipError_t launch_matvec_apply(hipStream_t s, int trans, int nleaf, int L, const int64_t* d_leaf_off,
                               const int32_t* d_rpre, int R, const S* D, int64_t ldd, const S* Ua, int64_t lda,
                               const double* X, int64_t ldx, const double* tree, double* Y, int64_t ldy, int nrhs, int full);

// Gradient pieces.  grad_leaf: dD_a = add_a - Lam_a X_a^T on the leaf blocks (add may be null).
// grad_gen: out(I_a, c) = add(I_a, c) - Left(I_a, :) S(c, :)^T with S the projection-tree entry of
// the sibling of a's ancestor at c's level; tri = 1 restricts the sum to the columns of the
// levels above c's level.
template <typename S>
hipError_t launch_grad_leaf(hipStream_t s, int nleaf, int m_max, const int64_t* d_leaf_off, int nrhs,
                            const double* X, int64_t ldx, const double* Lam, int64_t ldl, S* dD, int64_t ldd,
                            const double* add = nullptr, int64_t ldadd = 0);
template <typename S>
hipError_t launch_grad_gen(hipStream_t s, int nleaf, int L, const int64_t* d_leaf_off, const int32_t* d_rpre, int R,
                           int nrhs, const double* Left, int64_t ldl, const double* tree, S* out, int64_t ldo,
                           const double* add = nullptr, int64_t ldadd = 0, int tri = 0);

// Refinement helpers (FP64).
hipError_t launch_colnorms(hipStream_t s, int64_t n, int nrhs, const double* X, int64_t ldx, double* part,
                           double* out2, double* outinf);
template <typename T>
hipError_t launch_scale_down(hipStream_t s, int64_t n, int nrhs, const double* Rr, int64_t ldr, const double* sc,
                             T* out, int64_t ldo);
template <typename T>
hipError_t launch_axpy_up(hipStream_t s, int64_t n, int nrhs, const T* d, int64_t ldd, const double* sc, double* X,
                          int64_t ldx);
hipError_t launch_residual(hipStream_t s, int64_t n, int nrhs, const double* B, int64_t ldb, double* AX, int64_t ldax);
template <typename T, typename S>
hipError_t launch_convert(hipStream_t s, int64_t rows, int cols, const S* in, int64_t ldi, T* out, int64_t ldo,
                          int64_t gsi = 256);

}  // namespace hodlr

namespace hodlr {
// Fixed device scratch of the allocation-free solve (noalloc.hip): capacity in
// bytes, and this device's address of it (the current device; looked up once
// per device).
size_t scratch_capacity();
hipError_t scratch_device_ptr(void** out);
}  // namespace hodlr

namespace hodlr {
// Coupling factors of the levels that have them, for the log-determinant:
// per entry p < n, `count` parents of rank r, K stored with kp entries per
// parent from element kvoff of the K vectors (interchanges, 1 / pivots).
struct LogdetLevels {
  int n = 0;
  int count[HODLR_MAX_LEVELS];
  int r[HODLR_MAX_LEVELS];
  int kp[HODLR_MAX_LEVELS];
  int64_t kvoff[HODLR_MAX_LEVELS];
};
// log|det A| (out[0]) and its sign (out[1]) from the leaf factors (1 / U_jj,
// interchanges) and the coupling factors; item_log / item_par: nleaf + sum of
// counts scratch entries.
template <typename T>
hipError_t launch_logdet(hipStream_t s, int nleaf, int ldl, const int64_t* d_leaf_off, const T* udinv,
                         const int32_t* piv, const T* Kud, const int32_t* Kpiv, const LogdetLevels& lv,
                         double* item_log, int* item_par, double* out);
}  // namespace hodlr

namespace hodlr {
// Pieces of the gradient of log|det A| (logdet.hip).
template <typename S>
hipError_t launch_transpose_leaves(hipStream_t s, int nleaf, int m_max, const int64_t* d_leaf_off, const S* D,
                                   int64_t ldd, S* Dt, int64_t ldt);
template <typename T>
hipError_t launch_identity_leaves(hipStream_t s, int nleaf, int ncols, const int64_t* d_leaf_off, T* E, int64_t lde);
template <typename T>
hipError_t launch_identity_blocks(hipStream_t s, int nblk, int n2, T* X);
template <typename T>
hipError_t launch_pblocks(hipStream_t s, int nparents, int r, const T* Kinv, int64_t ldk, int64_t pstride, double* Pd);
hipError_t launch_node_mix(hipStream_t s, int64_t n, int L, int R, const int64_t* d_leaf_off, const int32_t* d_rpre,
                           const int64_t* d_pdoff, const double* Pd, int trans, const double* in, double* out);
}  // namespace hodlr

namespace hodlr {
// Construction by cross approximation (construct.hip).
struct ConstructKernel {
  int kind;
  int dim;
  const double* pts;
  int64_t ldp;
  const double* nrm;
  const double* w;
  const double* kap;
  double ell;
  double shift;
};
// One sibling block A(I_a, I_b): rows r0 .. r0 + m, columns c0 .. c0 + n, its
// generators in columns col .. col + rank of U_big / V_big, its tiles
// tile0 .. tile0 + ntile (each covers aca_tile_elems() rows and columns).
struct AcaBlock {
  int64_t r0, c0;
  int32_t m, n, col, rank, tile0, ntile;
};
struct AcaTile {
  int32_t blk, t, gtile;
};
// per-tile partial argmax of the residual rows (modulus, signed value, column)
// and columns (score, row); pivot rows [block][kmax]
struct AcaPartials {
  double* rp_abs;
  double* rp_val;
  int* rp_idx;
  double* cp_abs;
  int* cp_idx;
  int* piv;
};
int aca_tile_elems();
template <typename TS>
hipError_t launch_construct_leaves(hipStream_t s, const ConstructKernel& k, int nleaf, const int64_t* d_off, int m_max,
                                   TS* D, int64_t ldd);
// step `step` of every block (rank > step): the residual-row launch and the residual-column launch
hipError_t launch_aca_step(hipStream_t s, const ConstructKernel& k, int ntiles, const AcaBlock* blocks,
                           const AcaTile* tiles, int step, int kmax, double* U, int64_t ldu, double* V, int64_t ldv,
                           AcaPartials p);
template <typename TS>
hipError_t launch_store_cols(hipStream_t s, int64_t n, int ncols, const double* src, int64_t lds, TS* dst, int64_t ldd);
}  // namespace hodlr

namespace hodlr {
// Real embedding of complex matrices (embed.hip): E (2n x 2c, ld lde) =
// emb(M) for complex M (n x c, interleaved, ld ldm in complex elements), and
// back (M from the first column of each 2 x 2 block).
hipError_t launch_embed_cols(hipStream_t s, int64_t n, int ncols, const double* M, int64_t ldm, double* E, int64_t lde);
hipError_t launch_deembed_cols(hipStream_t s, int64_t n, int ncols, const double* E, int64_t lde, double* M,
                               int64_t ldm);
}  // namespace hodlr
