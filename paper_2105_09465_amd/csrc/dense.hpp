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

// In-place lower Cholesky of the n x n matrix A (column-major, lda >= n; only
// the lower triangle is read; the strict upper triangle is zeroed block by
// block). logd[n] receives ln of the factor's diagonal, *logdet (nullable) =
// ln|A|, *info = 0 or the first failing column + 1 (device scalars).
int dense_cholesky(rocblas_handle h, double* A, int n, int lda, double* logd, double* logdet, int* info,
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
