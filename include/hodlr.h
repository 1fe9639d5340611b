/*
 * hodlr.h — C ABI of the MI355X (gfx950) HODLR factor/solve library.
 *
 * Problem (paper: Section I, the linear system A x = b; Section III, eq.
 * "e:hxb"): A is an N x N HODLR matrix on a binary cluster tree T_L
 * (Definition "Cluster tree"): level l has 2^l nodes, each a consecutive
 * index set, siblings partition their parent.  A is given by
 *   - its 2^L leaf diagonal blocks D_a = A(I_a, I_a), and
 *   - low-rank generators for every sibling pair (a, b):
 *       A(I_a, I_b) = U_a V_b^T            (eq. "e:rank", real field).
 * The generators of all levels are concatenated into U_big / V_big
 * (Fig. "f:cat", eq. "e:u"): level l (1 <= l <= L, rank r_l) occupies
 * columns [R_{l-1}, R_l) with R_l = r_1 + ... + r_l, and node a's block is
 * rows I_a of those columns.  The leaf blocks are stacked into
 * D_big (Fig. "f:dk"): row block I_a, columns [0, |I_a|).
 *
 * Memory layout: every matrix argument is COLUMN-MAJOR with an explicit
 * leading dimension (element (i, j) at ptr[i + j*ld]).  Device pointers
 * unless marked "host".  Arguments are never freed by the library.
 *
 * Streams: every call is ordered on `stream` (a hipStream_t; NULL = the
 * null stream).  Calls that return a convergence or singularity verdict
 * synchronise `stream` once per verdict; all others are asynchronous.
 * A factorization keeps one solve workspace per stream it is used on, so
 * hodlr_solve, hodlr_solve_adjoint and hodlr_grad may run concurrently on
 * different streams (and from different host threads) on one factorization;
 * calls on one stream are ordered by the stream.  hodlr_refactor waits (on
 * the device) for the last call on every stream before it overwrites the
 * factors, and later calls wait for it.
 *
 * Errors: negative status = invalid argument / resource error, detected
 * before any kernel is launched where possible; nothing is written then.
 * Positive status = numerical verdict (see each call).
 */
#ifndef HODLR_H
#define HODLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HODLR_F64 = 0,   /* IEEE double                                      */
  HODLR_F32 = 1,   /* IEEE single                                      */
  HODLR_BF16 = 2,  /* bfloat16 MFMA operands, FP32 storage/accumulate  */
  HODLR_C128 = 3   /* complex double, (re, im) interleaved (storage only) */
} hodlr_dtype;

/* Complex matrices (the field F = C of the paper; A(I_a, I_b) = U_a V_b^*,
 * V^* the conjugate transpose).  A hodlr_matrix with dtype HODLR_C128 holds
 * D, U, V as interleaved complex doubles, leading dimensions counted in
 * complex elements.  hodlr_factor factors the real embedding of A: entry
 * p + i q becomes the real 2 x 2 block [[p, -q], [q, p]], and index i the rows
 * and columns 2i, 2i+1.  The embedding is a real HODLR matrix on the same tree,
 * with doubled leaf sizes (each leaf <= HODLR_MAX_LEAF / 2) and doubled ranks
 * (each r_l <= HODLR_MAX_RANK / 2), else HODLR_ERR_UNSUPPORTED.  The
 * factorization keeps its own embedded copy of D, U, V (the caller's arrays
 * are read once) and takes compute HODLR_F64, HODLR_F32 or HODLR_BF16 on it;
 * HODLR_INPLACE is unsupported.  On complex factors:
 *   - hodlr_solve and hodlr_solve_noalloc (trans = 0) take B as N x nrhs complex
 *     (interleaved, ldb in complex elements), which is the embedded real vector
 *     itself: B <- A^{-1} B;
 *   - hodlr_solve_adjoint and hodlr_solve_noalloc (trans = 1) give
 *     B <- A^{-*} B (emb(A)^T = emb(A^*));
 *   - refinement works as for real matrices, on the embedded copy;
 *   - hodlr_matvec on a complex matrix gives A X, or A^* X when trans = 1;
 *   - hodlr_factors_y writes the complex Y_big (N x R, ldy in complex elements);
 *   - hodlr_logdet gives log|det A| with *sign = 1 (0 when singular), because
 *     det emb(A) = |det A|^2 carries no phase;
 *   - hodlr_grad and hodlr_logdet_grad return HODLR_ERR_UNSUPPORTED.
 * The embedding costs twice the bytes and flops of native complex arithmetic. */

typedef enum {
  HODLR_OK = 0,
  HODLR_ERR_ARG = -1,          /* bad shape, pointer, rank or leading dimension */
  HODLR_ERR_ALLOC = -2,        /* device allocation failed                     */
  HODLR_ERR_HIP = -3,          /* a HIP runtime call failed                    */
  HODLR_ERR_UNSUPPORTED = -4,  /* valid but outside this build's limits        */
  HODLR_ERR_SINGULAR = 1,      /* an exactly zero pivot in a leaf or a K       */
  HODLR_ERR_NOT_CONVERGED = 2  /* iterative refinement did not reach tol       */
} hodlr_status;

/* Limits of this build. */
#define HODLR_MAX_LEAF 256     /* largest leaf block |I_a|                      */
#define HODLR_MAX_RANK 64      /* largest per-level rank r_l                    */
#define HODLR_MAX_LEVELS 24

/* Flags of hodlr_factor.
 * HODLR_INPLACE: the factorization overwrites the caller's matrix, as in
 *   Section III-B (the leaf LU factors replace D_big, Y_big replaces U_big):
 *   the leaf factors of leaf a go to rows I_a of D (ld ldd; needs
 *   |I_a| % 16 == 0 for every leaf), Y_big to U (column-major, ld ldu), and
 *   the factors need the storage type to be the compute type (F64 storage
 *   with F64, F32 storage with F32 or BF16).  D and U are then written, so
 *   refinement (opts->refine) and hodlr_grad, which need the original
 *   matrix, return HODLR_ERR_ARG on such a factorization.  V is only read.
 *   Without the flag D, U and V are only read and must outlive the factors. */
#define HODLR_INPLACE 1

/* A HODLR matrix (inputs of the factorization; Alg. "a:gpuf" "Require").
 *   n             N >= 1
 *   levels        L >= 0; the tree has 2^L leaves
 *   leaf_offsets  host, 2^L + 1 strictly increasing int64, [0] = 0, [2^L] = N;
 *                 node i of level l spans leaves [i 2^{L-l}, (i+1) 2^{L-l}).
 *                 NULL = uniform tree (requires 2^L | N).
 *   ranks         host, L entries, ranks[l-1] = r_l, 0 <= r_l <= HODLR_MAX_RANK
 *                 and r_l <= size of every level-l node (else HODLR_ERR_ARG).
 *                 May be NULL if L = 0.
 *   dtype         storage type of D, U, V: HODLR_F64, HODLR_F32 or HODLR_C128
 *                 (complex, see "Complex matrices" above)
 *   D, ldd        N x m_max (m_max = largest leaf), ldd >= N
 *   U, ldu        N x R (R = R_L), ldu >= N (ignored if R = 0)
 *   V, ldv        N x R, ldv >= N
 * The library only reads D, U, V (unless hodlr_factor is given
 * HODLR_INPLACE).  A factorization keeps referring to them (refinement
 * residuals and gradients), so they must outlive it unchanged. */
typedef struct {
  int64_t n;
  int32_t levels;
  const int64_t *leaf_offsets;
  const int32_t *ranks;
  hodlr_dtype dtype;
  const void *D;
  int64_t ldd;
  const void *U;
  int64_t ldu;
  const void *V;
  int64_t ldv;
} hodlr_matrix;

/* Opaque factorization (Alg. "a:gpuf" "Ensure": Y_big, the block LU
 * factorizations of D_big^L and of K_big^0 .. K_big^{L-1}).  Owns its
 * device memory; immutable after hodlr_factor except by hodlr_refactor. */
typedef struct hodlr_factors hodlr_factors;

/* First exactly-zero pivot, in factorization order (leaves first, then the
 * coupling matrices from level L-1 up to 0).  level = L for a leaf (node =
 * leaf index), else the parent level of the K; column is 0-based. */
typedef struct {
  int32_t level;
  int32_t column;
  int64_t node;
} hodlr_info;

/* Solve options.  refine = 0: one application of the stored factors in the
 * factorization's precision.  refine = 1: FP64 iterative refinement around
 * the factors, with an FP64 residual b - A x evaluated from the original
 * D, U, V; stops when max over columns ||b - A x||_2 / ||b||_2 <= tol, fails
 * with HODLR_ERR_NOT_CONVERGED after max_iter steps or when the residual
 * grows on two consecutive steps. */
typedef struct {
  int32_t refine;
  int32_t max_iter;
  double tol;
} hodlr_solve_opts;

typedef struct {
  int32_t iters;      /* refinement steps taken (0 without refinement)       */
  int32_t converged;  /* 1 if relres <= tol                                   */
  double relres;      /* final max-column relative residual (refine only)    */
} hodlr_solve_stats;

/* Factorization (Section III-B Alg. "a:fact" / Section III-C Alg. "a:gpuf"):
 * batched LU with partial pivoting of every leaf, Y_big = D^{-1} U_big on all
 * columns, then for l = L-1 .. 0: the coupling products V^T Y, the LU of
 * K_g = [[V_a^T Y_a, I], [I, V_b^T Y_b]] (eq. "e:k") and the update of
 * Y_big(:, 1:R_l) (eqs. "e:node1", "e:node2").
 *   A        the matrix (see hodlr_matrix)
 *   compute  HODLR_F64 (requires dtype F64), HODLR_F32 or HODLR_BF16.  F32
 *            and BF16 keep FP32 factors (leaf LU, Y_big, K); BF16 rounds the
 *            operands of the matrix-core products to bfloat16 with FP32
 *            accumulation (the leaf LU's trailing updates, the leaf solve on
 *            U_big and the coupling products and updates V^T Y, Y W), while
 *            the pivot searches, the panels and the coupling matrices K stay
 *            FP32.  Solves with F32/BF16 factors run in FP32; opts->refine
 *            recovers FP64 accuracy.
 *   flags    0 or HODLR_INPLACE (other bits: HODLR_ERR_ARG)
 *   F        out: new factorization object (NULL on negative status)
 * Returns HODLR_ERR_SINGULAR (factors kept but unusable; *info filled if
 * info != NULL) when a pivot is exactly zero.  Synchronises the stream once
 * (singularity verdict).  Allocates device memory (hipMalloc). */
hodlr_status hodlr_factor(const hodlr_matrix *A, hodlr_dtype compute, int32_t flags, void *stream,
                          hodlr_factors **F, hodlr_info *info);

/* Recompute the factorization in F's storage for new values of D, U, V
 * with exactly the same tree, ranks, storage type and leading dimensions
 * (pointers may change; an in-place factorization then overwrites the new
 * D and U).  Allocates nothing.  Same verdicts as hodlr_factor.  Must not be
 * called from one host thread while another host thread calls into F. */
hodlr_status hodlr_refactor(hodlr_factors *F, const hodlr_matrix *A, void *stream, hodlr_info *info);

/* Solution (Alg. "a:solve" / Alg. "a:gpus"): B <- A^{-1} B in place
 * (x overwrites b).  B is N x nrhs FP64, ldb >= N, nrhs >= 0.  With
 * opts == NULL or refine == 0 the solve runs in the factors' precision.
 * st may be NULL. */
hodlr_status hodlr_solve(const hodlr_factors *F, int64_t nrhs, double *B, int64_t ldb,
                         const hodlr_solve_opts *opts, void *stream, hodlr_solve_stats *st);

/* Adjoint solution B <- A^{-T} B on the same factors.  Uses the product
 * form of Section III-E (A = D F_L ... F_1, each F a 2x2 block factor that
 * eq. "e:wood" inverts): A^{-T} = D^{-T} F_L^{-T} ... F_1^{-T}, applied top
 * level first with transposed coupling solves, leaf solves last.
 * Refinement (opts->refine) uses the FP64 residual with A^T. */
hodlr_status hodlr_solve_adjoint(const hodlr_factors *F, int64_t nrhs, double *B, int64_t ldb,
                                 const hodlr_solve_opts *opts, void *stream, hodlr_solve_stats *st);

/* Allocation-free variant of hodlr_solve / hodlr_solve_adjoint without
 * refinement, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * B <- A^{-1} B (trans = 0) or A^{-T} B (trans = 1), B N x nrhs FP64,
 * ldb >= N, in the factors' precision, with the same kernels and results as
 * hodlr_solve / hodlr_solve_adjoint with refine = 0.  Instead of a per-stream
 * workspace the call uses a fixed 64 MiB device scratch array that the
 * library holds once per GPU until the process ends; it calls no hipMalloc,
 * hipFree or allocating routine.  hodlr_solve_noalloc_bytes(F, nrhs) gives
 * the scratch bytes a call needs; a call needing more than 64 MiB returns
 * HODLR_ERR_ARG before launching anything (so does a call from a device
 * other than the one F was factored on, which must be the current device).
 * Every such call on one GPU shares that GPU's scratch, whose contents the
 * last call leaves behind (nothing in it needs to start at zero): calls that
 * may overlap on one GPU (other streams, other factorizations) race and must
 * be ordered by the caller.  hodlr_refactor and hodlr_destroy wait for the
 * last such call on F.  No refinement: its per-step convergence test
 * synchronises the stream. */
hodlr_status hodlr_solve_noalloc(const hodlr_factors *F, int32_t trans, int64_t nrhs, double *B,
                                 int64_t ldb, void *stream);
size_t hodlr_solve_noalloc_bytes(const hodlr_factors *F, int64_t nrhs);

/* FP64 matrix product Y = A X (trans = 0) or Y = A^T X (trans = 1), reading
 * D, U, V in their storage type: y_a = D_a x_a + sum over levels of
 * U_a (V_b^T x_b) for the sibling b of each ancestor-or-self a (eq. "e:rank").
 * X: N x nrhs (ldx >= N), Y: N x nrhs (ldy >= N); X and Y must not overlap.
 * Allocates temporary device memory. */
hodlr_status hodlr_matvec(const hodlr_matrix *A, int32_t trans, int64_t nrhs, const double *X,
                          int64_t ldx, double *Y, int64_t ldy, void *stream);

/* Gradients of a scalar loss through x = A^{-1} b, given the solution X and
 * the adjoint Lambda = A^{-T} dL/dx (both N x nrhs FP64): dL/dA = -Lambda X^T
 * restricted to the HODLR parameters,
 *   dD_a = -Lambda_a X_a^T, dU_a = -Lambda_a (V_b^T X_b)^T, dV_b = -X_b (U_a^T Lambda_a)^T.
 * dD, dU, dV are written in the storage type and layout of F's D, U, V
 * (N x m_max with ldd, N x R with ldu / ldv); entries of dD outside the
 * leaf blocks are left untouched. */
hodlr_status hodlr_grad(const hodlr_factors *F, int64_t nrhs, const double *X, int64_t ldx,
                        const double *Lambda, int64_t ldl, void *dD, void *dU, void *dV,
                        void *stream);

/* Copy Y_big (N x R; level-l columns at rows I_a hold Y_a = A_a^{-1} U_a,
 * eq. "e:recursion") into Y as FP64 (ldy >= N). */
hodlr_status hodlr_factors_y(const hodlr_factors *F, double *Y, int64_t ldy, void *stream);

/* Sign and natural logarithm of |det A| from the stored factors (Section
 * III-E, "Determinant"): A = D F_L ... F_1, so det A is the product of the
 * leaf determinants and of det F_g over the parents g, and by Sylvester's
 * determinant theorem det F_g = (-1)^r det K_g (K_g of eq. "e:k" is the
 * 2x2 block factor's small matrix with its two row blocks exchanged).  Each
 * determinant is the product of its LU pivots with the sign of its
 * interchanges.  Host outputs: *sign in {-1, 0, +1} (0 when a pivot is
 * exactly zero, *logabs then -inf), *logabs summed in FP64 in a fixed order
 * (deterministic).  For F32/BF16 factors the pivots are FP32.  Synchronises
 * `stream` once. */
hodlr_status hodlr_logdet(const hodlr_factors *F, double *sign, double *logabs, void *stream);

/* Gradient of log|det A| with respect to the HODLR parameters (Section III-E
 * "Determinant" differentiated): by Jacobi's formula the gradient with
 * respect to A is A^{-T}, restricted here to the parameters through
 * A(I_a, I_a) = D_a and A(I_a, I_b) = U_a V_b^T:
 *   dD_a = (A^{-T})_aa,  dU_a = (A^{-T})_ab V_b,  dV_b = ((A^{-T})_ab)^T U_a.
 * Computed through the factorization, never forming A^{-1}: with
 * T_a = V_a^T Y_a and P_a the a-block of K_g^{-1} (g the parent of a),
 * log|det A| = sum log|det D| + sum log|det K|, so
 *   dD_a = D_a^{-T} - Lam(I_a, :) Y(I_a, :)^T,
 *   dU_m = Lam(I_m, c_l) - Lam(I_m, 1:R_{l-1}) Y(I_n, 1:R_{l-1})^T V_n,
 *   dV_n = Y(I_n, c_l) P_n - Y(I_n, 1:R_{l-1}) Lam(I_m, 1:R_{l-1})^T U_m
 * for siblings (m, n) of level l, where Lam(I_a, c_l) = A_a^{-T} V_a P_a^T
 * comes from Y_big of A^T (a second factorization, of D^T with U and V
 * exchanged).  dD, dU, dV are written in the storage type and layout of F's
 * D, U, V (as hodlr_grad).  Arithmetic: the factors' precision for the
 * solves, FP64 for the assembly.  Needs the original D, U, V
 * (HODLR_ERR_ARG on in-place factors), HODLR_ERR_SINGULAR on a singular
 * factorization.  Allocates temporaries (two FP64 projection trees of
 * (2^{L+1} - 2) R^2 entries, four N x R FP64 blocks, the factors of A^T) and
 * synchronises `stream` before freeing them. */
hodlr_status hodlr_logdet_grad(const hodlr_factors *F, void *dD, void *dU, void *dV, void *stream);

/* Kernel matrices that hodlr_construct compresses.  Entry A(p, q), p != q:
 *   HODLR_KERNEL_GAUSS       exp(-|x_p - x_q|^2 / (2 ell^2))          (Section I,
 *   HODLR_KERNEL_MATERN32    (1 + s) exp(-s), s = sqrt(3) |x_p - x_q| / ell
 *                            "Kernel matrices": Gaussian and Matern kernels)
 *   HODLR_KERNEL_LAPLACE_DL  w_q n_q . (x_p - x_q) / (2 pi |x_p - x_q|^2)
 *                            (Section IV-B, the double-layer kernel d(x, y) of
 *                            eq. "e:laplace_int" with trapezoidal weights w_q
 *                            and unit normals n_q of a closed curve in 2-D)
 * Diagonal A(p, p): 1 (radial kernels) or the smooth limit w_p kappa_p / (4 pi)
 * (double layer, kappa the signed curvature), plus `shift` (a nugget, or 1/2
 * for the second-kind equation).
 *   points     device, N x dim FP64, column-major with ld ldp (dim 1..3 for the
 *              radial kernels, 2 for the double layer)
 *   normals    LAPLACE_DL: device, N x 2 FP64 with ld ldp; else ignored
 *   weights, curvature   LAPLACE_DL: device, N FP64 each; else ignored
 *   ell        length scale of the radial kernels, > 0
 */
typedef enum {
  HODLR_KERNEL_GAUSS = 0,
  HODLR_KERNEL_MATERN32 = 1,
  HODLR_KERNEL_LAPLACE_DL = 2
} hodlr_kernel_kind;

typedef struct {
  hodlr_kernel_kind kind;
  int32_t dim;
  const double *points;
  int64_t ldp;
  const double *normals;
  const double *weights;
  const double *curvature;
  double ell;
  double shift;
} hodlr_kernel;

/* Construction of a HODLR approximation of the kernel matrix of `k`
 * (Section II-B: every sibling block compressed on its own; Section IV-A
 * compresses them by an approximate partial-pivoted LU).  The leaf blocks
 * are exact; every sibling block A(I_a, I_b) of level l is approximated by
 * r_l steps of cross approximation with partial pivoting:
 *   v = A(i_k, :) - sum_{l<k} u_l(i_k) v_l,  j_k = argmax |v|,  v_k = v / v(j_k),
 *   u_k = A(:, j_k) - sum_{l<k} v_l(j_k) u_l,  i_{k+1} = argmax over unused rows |u_k|,
 * i_1 the block's first row, ties to the lowest index, an exhausted step
 * (v(j_k) = 0) giving u_k = v_k = 0; U_a = [u_1..u_r] and V_b = [v_1..v_r].
 * The tree, ranks and outputs are described as in hodlr_matrix: n, levels,
 * leaf_offsets (host, NULL = uniform), ranks (host), dtype (F64 or F32
 * storage of the outputs), D (N x m_max, ld ldd; entries right of a leaf's
 * width set to zero), U, V (N x R, ld ldu / ldv; every entry written).
 * Arithmetic is FP64 throughout; F32 outputs are rounded once at the end.
 * N < 2^31.  Allocates temporaries (pivot bookkeeping; FP64 copies of U, V
 * for F32 outputs) and synchronises `stream` before freeing them. */
hodlr_status hodlr_construct(const hodlr_kernel *k, int64_t n, int32_t levels, const int64_t *leaf_offsets,
                             const int32_t *ranks, hodlr_dtype dtype, void *D, int64_t ldd, void *U,
                             int64_t ldu, void *V, int64_t ldv, void *stream);

/* Device bytes owned by F: the factors, the factorization's workspace and
 * the solve workspaces of every stream F was used on. */
size_t hodlr_factor_bytes(const hodlr_factors *F);

/* Release F.  Waits for F's own pending work only (the factorization and
 * the last call on each stream that used F), not for the whole device.
 * NULL is ignored. */
void hodlr_destroy(hodlr_factors *F);

const char *hodlr_status_string(hodlr_status s);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel of the library.  enable = 1 starts recording (clears totals),
 * 0 stops.  hodlr_kernel_times fills up to `cap` entries: names[i] (static
 * strings), total milliseconds and launch counts; returns the number of
 * kernels seen.  Synchronises the recorded streams. */
void hodlr_timing_enable(int32_t enable);
int32_t hodlr_kernel_times(const char **names, double *total_ms, int64_t *launches, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* HODLR_H */
