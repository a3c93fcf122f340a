// Dense FP64 helpers of the preconditioner (csrc/dense.hip).
#pragma once

#include <rocblas/rocblas.h>

#include "common.hpp"

namespace gpl {

// rocBLAS handle of this host thread on the current device (two per device:
// slot 0 and slot 1, for work on two streams at once), set to `stream`, host
// pointer mode, and the given scratch memory (rocBLAS allocates none).
int blas_handle(rocblas_handle* out, hipStream_t stream, void* scratch, size_t scratch_bytes, int slot = 0);

// 1 / sqrt(v) for a positive normal v to FP64 accuracy: the hardware estimate
// refined by two Newton steps r <- r + r (1 - v r^2) / 2 (each about doubles
// the number of correct bits).
__device__ __forceinline__ double rsqrt_f64(double v) {
  double r = __builtin_amdgcn_rsq(v);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-(v * r), r, 1.0);
    r = fma(0.5 * r, e, r);
  }
  return r;
}

// A second stream of this host thread on the current device (non-blocking,
// default priority) and three events for ordering it against the caller's
// stream, created on first use and kept.
int side_stream(hipStream_t* s, hipEvent_t ev[3]);

// Scratch memory handed to rocBLAS by every call that uses it.
constexpr size_t kBlasScratch = size_t(32) << 20;

// Inverse and log-determinant of the symmetric positive definite k x k matrix
// G + shift I (k a multiple of 64) by bordering, one block of 64 rows at a
// time: with Ginv the inverse of the leading block A already formed, the next
// 64 rows B and diagonal block C give Y = B A^{-1}, the Schur complement
// S = C - Y B^T (its Cholesky factor D and D^{-1} in one workgroup),
// W = D^{-1} Y and
//   inverse = [[A^{-1} + W^T W, -(D^{-T} W)^T], [-D^{-T} W, S^{-1}]],
//   ln|G| = ln|A| + ln|S|.
// G is column-major (ldg). border_step(j0) reads columns j0 .. j0 + 63 of G
// down to row j0 + 63 (the diagonal block from its lower triangle) and the
// inverse of the leading j0 x j0 block left in place by the earlier steps, and
// writes the inverse of the leading (j0 + 64) block in place (both triangles);
// later columns are neither read nor written, so they may be filled in while
// earlier steps run. border_begin sets *info = 0; a step sets it (if still 0) to 1 + the index
// of the first pivot of its diagonal block that was not positive (the inverse is
// then meaningless); border_finish writes *logdet = ln|G + shift I| (the blocks'
// parts summed in a fixed order).
// Scratch (device, doubles): Y and W 64 x k, T and Dinv 64 x 64, ld_part k / 64,
// split for the split products (split_elems doubles, at least 64 x k).
struct SpdScratch {
  double *Y, *W, *T, *Dinv, *ld_part, *split;
  size_t split_elems;
};
int border_begin(int* info, hipStream_t stream);
int border_step(rocblas_handle h, double* G, int ldg, int j0, double shift, const SpdScratch& w, int* info,
                hipStream_t stream);
int border_finish(int k, const SpdScratch& w, double* logdet, hipStream_t stream);

// C (m x n) = alpha op(A) op(B) + beta C with the reduction dimension kdim
// split into nsplit parts (rocBLAS strided-batched products into scratch, then
// a sum in split order): GEMMs with one short side use the whole device this
// way. scratch: split_gemm_scratch(m, n, nsplit) bytes; scratch_elems is the
// number of doubles it holds, and nsplit is lowered to what fits (an error if
// not even one split does). With Cf set, the beta term reads C's entry (i, j)
// from Cf[i * n + j] as a float (C transposed and narrower) instead of from C.
size_t split_gemm_scratch(int m, int n, int nsplit);
int split_gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int kdim, int nsplit,
               double alpha, const double* A, int lda, const double* B, int ldb, double beta, double* C, int ldc,
               double* scratch, size_t scratch_elems, hipStream_t stream, const float* Cf = nullptr);

}  // namespace gpl
