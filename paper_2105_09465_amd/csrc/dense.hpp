// Dense FP64 helpers of the preconditioner (csrc/dense.hip).
#pragma once

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "common.hpp"

namespace gpl {

// rocBLAS handle of this host thread on the current device, set to `stream`,
// host pointer mode, and the given scratch memory (rocBLAS allocates none).
int blas_handle(rocblas_handle* out, hipStream_t stream, void* scratch, size_t scratch_bytes);

// Scratch memory handed to rocBLAS by every call that uses it.
constexpr size_t kBlasScratch = size_t(32) << 20;

// Scratch memory of the handle for the dense factorisations of the
// preconditioner (rocSOLVER's Cholesky and inverse of a matrix of the rank's
// size take their device memory from it).
constexpr size_t kSolverScratch = size_t(256) << 20;

// In-place lower Cholesky of the n x n matrix A (column-major, lda >= n; only
// the lower triangle is read and written) by rocSOLVER, then, with `inverse`,
// the lower triangle of A^{-1} in its place. logd[n] receives ln of the factor's
// diagonal, *logdet (nullable) = ln|A| summed from it in index order, *info = 0
// or the order of the first non-positive leading minor (device scalars).
int dense_cholesky(rocblas_handle h, double* A, int n, int lda, double* logd, double* logdet, int* info, bool inverse,
                   hipStream_t stream);

// B (m x 64, column-major, ld ldb) = B R^{-T} in place for the lower 64 x 64
// factor R (column-major, ld 64): each row solves x R^T = b by forward
// substitution, one row per thread, R in LDS.
int trsm_rows64(int m, const double* R, double* B, int ldb, hipStream_t stream);

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
