// Dense FP64 helpers of the preconditioner (csrc/dense.hip).
#pragma once

#include <rocblas/rocblas.h>

#include "common.hpp"

namespace gpl {

// rocBLAS handle of this host thread on the current device, set to `stream`,
// host pointer mode, and the given scratch memory (rocBLAS allocates none).
int blas_handle(rocblas_handle* out, hipStream_t stream, void* scratch, size_t scratch_bytes);

// Scratch memory handed to rocBLAS by every call that uses it.
constexpr size_t kBlasScratch = size_t(32) << 20;

// Inverse and log-determinant of a symmetric positive definite k x k matrix
// (k a multiple of 64) by bordering: with Ginv the inverse of the leading
// block A already formed, the next 64 rows B and diagonal block C give
// Y = B A^{-1}, the Schur complement S = C - Y B^T (its Cholesky factor D and
// D^{-1} in one workgroup), W = D^{-1} Y and
//   inverse = [[A^{-1} + W^T W, -(D^{-T} W)^T], [-D^{-T} W, S^{-1}]],
//   ln|G| = ln|A| + ln|S|.
// G (column-major, ldg) is read from its lower triangle and receives the whole
// inverse in place (both triangles); *logdet = ln|G| (the blocks' parts summed
// in a fixed order); *info = 0, or 1 + the index of the first pivot of a
// diagonal block that was not positive (the inverse is then meaningless).
// Scratch (device, doubles): Y and W 64 x k, T and Dinv 64 x 64, ld_part k / 64,
// split for the split products (split_elems doubles, at least 64 x k).
struct SpdScratch {
  double *Y, *W, *T, *Dinv, *ld_part, *split;
  size_t split_elems;
};
int spd_inverse(rocblas_handle h, double* G, int k, int ldg, const SpdScratch& w, double* logdet, int* info,
                hipStream_t stream);

// C (m x n) = alpha op(A) op(B) + beta C with the reduction dimension kdim
// split into nsplit parts (rocBLAS strided-batched products into scratch, then
// a sum in split order): GEMMs with one short side use the whole device this
// way. scratch: split_gemm_scratch(m, n, nsplit) bytes; scratch_elems is the
// number of doubles it holds, and nsplit is lowered to what fits (an error if
// not even one split does).
size_t split_gemm_scratch(int m, int n, int nsplit);
int split_gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int kdim, int nsplit,
               double alpha, const double* A, int lda, const double* B, int ldb, double beta, double* C, int ldc,
               double* scratch, size_t scratch_elems, hipStream_t stream);

}  // namespace gpl
