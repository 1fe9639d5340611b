// Complex HODLR matrices through the real embedding (the field F = C of the
// paper; A(I_a, I_b) = U_a V_b^*, eq. "e:rank").  A complex entry p + i q
// becomes the real 2 x 2 block [[p, -q], [q, p]] and index i the rows (and
// columns) 2i, 2i+1.  The embedding maps products to products and M^* to
// emb(M)^T, so emb(A) is a real HODLR matrix on the same tree with doubled
// leaf sizes and ranks, U~ = emb(U_big), V~ = emb(V_big) (U~ V~^T = emb(U V^*)),
// and a complex vector stored as interleaved (re, im) pairs is already the
// embedded real vector: emb(A) x~ is A x in the same storage.
#include "internal.h"

namespace hodlr {

namespace {
constexpr int kEmThreads = 256;
}

// E (2n x 2c, ld lde) = emb(M) for M complex n x c (interleaved, ld ldm complex elements)
__global__ __launch_bounds__(kEmThreads) void embed_cols_kernel(int64_t n, const double* __restrict__ M, int64_t ldm,
                                                                double* __restrict__ E, int64_t lde) {
  const int64_t i = (int64_t)blockIdx.x * kEmThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t c = blockIdx.y;
  const double re = M[2 * (i + c * ldm)];
  const double im = M[2 * (i + c * ldm) + 1];
  double* e0 = E + 2 * i + (2 * c) * lde;  // column 2c: (re, im)
  double* e1 = e0 + lde;                   // column 2c + 1: (-im, re)
  e0[0] = re;
  e0[1] = im;
  e1[0] = -im;
  e1[1] = re;
}

// M (complex n x c, ld ldm) from the first column of each 2 x 2 block of E (2n x 2c, ld lde)
__global__ __launch_bounds__(kEmThreads) void deembed_cols_kernel(int64_t n, const double* __restrict__ E, int64_t lde,
                                                                  double* __restrict__ M, int64_t ldm) {
  const int64_t i = (int64_t)blockIdx.x * kEmThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t c = blockIdx.y;
  const double* e0 = E + 2 * i + (2 * c) * lde;
  M[2 * (i + c * ldm)] = e0[0];
  M[2 * (i + c * ldm) + 1] = e0[1];
}

hipError_t launch_embed_cols(hipStream_t s, int64_t n, int ncols, const double* M, int64_t ldm, double* E,
                             int64_t lde) {
  if (n == 0 || ncols == 0) return hipSuccess;
  if (ncols > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(embed_cols_kernel, dim3((unsigned)((n + kEmThreads - 1) / kEmThreads), ncols), dim3(kEmThreads),
                     0, s, n, M, ldm, E, lde);
  return hipGetLastError();
}

hipError_t launch_deembed_cols(hipStream_t s, int64_t n, int ncols, const double* E, int64_t lde, double* M,
                               int64_t ldm) {
  if (n == 0 || ncols == 0) return hipSuccess;
  if (ncols > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(deembed_cols_kernel, dim3((unsigned)((n + kEmThreads - 1) / kEmThreads), ncols),
                     dim3(kEmThreads), 0, s, n, E, lde, M, ldm);
  return hipGetLastError();
}

}  // namespace hodlr
