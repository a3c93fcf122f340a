// Dense FP64 linear algebra on small blocks for the preconditioner: a rocBLAS
// handle per host thread and device (its scratch memory always taken from the
// caller's workspace), and a blocked right-looking Cholesky factorisation: a
// one-workgroup kernel factors each 64 x 64 diagonal block in LDS, rocBLAS
// dtrsm forms the panel below it and dsyrk updates the trailing matrix. The
// log-determinant is summed from the factor's diagonal in a fixed order.
#include <cmath>

#include "common.hpp"
#include "dense.hpp"

namespace gpl {

static thread_local rocblas_handle t_handle[16] = {};

int blas_handle(rocblas_handle* out, hipStream_t stream, void* scratch, size_t scratch_bytes) {
  int dev = 0;
  GPL_HIP(hipGetDevice(&dev));
  GPL_REQUIRE(dev >= 0 && dev < 16, "device index %d out of range for the BLAS handles", dev);
  if (t_handle[dev] == nullptr) {
    if (rocblas_create_handle(&t_handle[dev]) != rocblas_status_success) {
      set_error("rocblas_create_handle failed");
      return GPL_EHIP;
    }
  }
  rocblas_handle h = t_handle[dev];
  if (rocblas_set_stream(h, stream) != rocblas_status_success ||
      rocblas_set_workspace(h, scratch, scratch_bytes) != rocblas_status_success ||
      rocblas_set_pointer_mode(h, rocblas_pointer_mode_host) != rocblas_status_success) {
    set_error("rocblas handle set-up failed");
    return GPL_EHIP;
  }
  *out = h;
  return GPL_OK;
}

// Factor the jb x jb diagonal block at A (leading dimension lda) in place:
// lower Cholesky by one wave in LDS, lane a owning row a (right-looking: after
// each column the lanes below it update their own rows). A non-positive or
// non-finite pivot sets *info to its global column + 1 (first one wins) and
// leaves the block unfinished. logd[c] = ln of the diagonal entry of column c.
constexpr int kDiag = 64;
__global__ __launch_bounds__(64) void potf2_kernel(double* A, int lda, int jb, int col0, double* logd, int* info) {
  // T[j][a] holds entry (a, j): lane a walks its row along j at consecutive
  // LDS addresses across the lanes (no bank conflicts)
  __shared__ double T[kDiag][kDiag + 1];
  __shared__ double ld[kDiag];  // written to logd after the loop (a global store before each barrier would
                                // make every barrier wait for it)
  const int a = threadIdx.x;
  for (int j = 0; j < jb; ++j)
    if (a < jb) T[j][a] = A[(size_t)j * lda + a];
  __syncthreads();
  for (int c = 0; c < jb; ++c) {
    const double p = T[c][c];
    if (!(p > 0.0) || !isfinite(p)) {
      if (a == 0) atomicCAS(info, 0, col0 + c + 1);
      return;
    }
    const double piv = sqrt(p);
    __syncthreads();
    if (a == c) {
      T[c][c] = piv;
      ld[c] = 0.5 * log(p);
    }
    double l = 0.0;
    if (a > c && a < jb) {
      l = T[c][a] / piv;
      T[c][a] = l;
    }
    __syncthreads();
    if (a > c && a < jb)
      for (int j = c + 1; j <= a; ++j) T[j][a] -= l * T[c][j];
    __syncthreads();
  }
  for (int j = 0; j < jb; ++j)
    if (a < jb) A[(size_t)j * lda + a] = j <= a ? T[j][a] : 0.0;
  if (a < jb) logd[col0 + a] = ld[a];
}

// out[0] = sum of logd[0..n) in index order (one wave, lane-strided then a
// butterfly), times two: ln|A| of the factored matrix.
__global__ void logdet_fold_kernel(int n, const double* logd, double* out) {
  const double s = wave_fold_sum(logd, n);
  if (threadIdx.x == 0) *out = 2.0 * s;
}

__global__ void zero_int_kernel(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

int dense_cholesky(rocblas_handle h, double* A, int n, int lda, double* logd, double* logdet, int* info,
                   hipStream_t stream) {
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, stream, info);
  GPL_LAUNCH_CHECK();
  const double one = 1.0, minus_one = -1.0;
  for (int j0 = 0; j0 < n; j0 += kDiag) {
    const int jb = std::min(kDiag, n - j0);
    double* Ajj = A + (size_t)j0 * lda + j0;
    hipLaunchKernelGGL(potf2_kernel, dim3(1), dim3(kDiag), 0, stream, Ajj, lda, jb, j0, logd, info);
    GPL_LAUNCH_CHECK();
    const int m = n - j0 - jb;
    if (m <= 0) break;
    double* Aij = Ajj + jb;  // the panel below the diagonal block
    if (rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                      rocblas_diagonal_non_unit, m, jb, &one, Ajj, lda, Aij, lda) != rocblas_status_success) {
      set_error("rocblas_dtrsm failed (n=%d, column %d)", n, j0);
      return GPL_EHIP;
    }
    double* Att = A + (size_t)(j0 + jb) * lda + (j0 + jb);
    if (rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, m, jb, &minus_one, Aij, lda, &one, Att, lda) !=
        rocblas_status_success) {
      set_error("rocblas_dsyrk failed (n=%d, column %d)", n, j0);
      return GPL_EHIP;
    }
  }
  if (logdet) {
    hipLaunchKernelGGL(logdet_fold_kernel, dim3(1), dim3(64), 0, stream, n, logd, logdet);
    GPL_LAUNCH_CHECK();
  }
  return GPL_OK;
}

// C (m x n, ld ldc) = alpha * sum_s Wp[s] + beta C, the splits in order.
__global__ void split_sum_kernel(int m, int n, int nsplit, const double* __restrict__ Wp, double alpha, double beta,
                                 double* C, int ldc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int r = e % m, c = e / m;
  double v = 0.0;
  for (int s = 0; s < nsplit; ++s) v += Wp[(size_t)s * m * n + e];
  double* y = C + (size_t)c * ldc + r;
  *y = beta == 0.0 ? alpha * v : alpha * v + beta * *y;
}

size_t split_gemm_scratch(int m, int n, int nsplit) { return (size_t)nsplit * m * n * sizeof(double); }

int split_gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int kdim, int nsplit,
               double alpha, const double* A, int lda, const double* B, int ldb, double beta, double* C, int ldc,
               double* scratch, size_t scratch_elems, hipStream_t stream) {
  const size_t per = (size_t)m * n;
  GPL_REQUIRE(m > 0 && n > 0 && kdim > 0, "split product of empty size");
  GPL_REQUIRE(scratch_elems >= per, "split product scratch holds %zu doubles, one split needs %zu", scratch_elems,
              per);
  const size_t fit = scratch_elems / per;
  nsplit = std::max(1, std::min(std::min(nsplit, kdim), (int)std::min<size_t>(fit, 1 << 20)));
  const int kc = cdiv(kdim, nsplit);
  nsplit = cdiv(kdim, kc);
  const int last = kdim - (nsplit - 1) * kc;  // rows of the reduction in the last split
  // element (i, l) of op(A) is A[l*lda + i] without transpose, A[i*lda + l] with it:
  // a split of the reduction index l moves A by kc columns (no transpose) or
  // kc rows (transpose); likewise for B with (l, j)
  const rocblas_stride sa = ta == rocblas_operation_none ? (rocblas_stride)kc * lda : kc;
  const rocblas_stride sb = tb == rocblas_operation_none ? kc : (rocblas_stride)kc * ldb;
  const double one = 1.0, zero = 0.0;
  if (nsplit > 1 &&
      rocblas_dgemm_strided_batched(h, ta, tb, m, n, kc, &one, A, lda, sa, B, ldb, sb, &zero, scratch, m,
                                    (rocblas_stride)m * n, nsplit - 1) != rocblas_status_success) {
    set_error("rocblas_dgemm_strided_batched failed");
    return GPL_EHIP;
  }
  if (rocblas_dgemm(h, ta, tb, m, n, last, &one, A + (size_t)(nsplit - 1) * sa, lda, B + (size_t)(nsplit - 1) * sb,
                    ldb, &zero, scratch + (size_t)(nsplit - 1) * m * n, m) != rocblas_status_success) {
    set_error("rocblas_dgemm (last split) failed");
    return GPL_EHIP;
  }
  hipLaunchKernelGGL(split_sum_kernel, dim3(cdiv(m * n, 256)), dim3(256), 0, stream, m, n, nsplit, scratch, alpha,
                     beta, C, ldc);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl
