// Dense FP64 linear algebra for the preconditioner: a rocBLAS handle per host
// thread and device (its scratch memory always taken from the caller's
// workspace), the Cholesky factor and inverse of a dense matrix by rocSOLVER
// (the log-determinant summed from the factor's diagonal in a fixed order), a
// row-parallel triangular solve with a 64 x 64 factor, and GEMMs with a long
// reduction split over the device.
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

// logd[c] = ln A[c][c] of a factor's diagonal.
__global__ void diag_log_kernel(int n, const double* __restrict__ A, int lda, double* logd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) logd[c] = log(A[(size_t)c * lda + c]);
}

// out[0] = sum of logd[0..n) in index order (one wave, lane-strided then a
// butterfly), times two: ln|A| of the factored matrix.
__global__ void logdet_fold_kernel(int n, const double* logd, double* out) {
  const double s = wave_fold_sum(logd, n);
  if (threadIdx.x == 0) *out = 2.0 * s;
}

int dense_cholesky(rocblas_handle h, double* A, int n, int lda, double* logd, double* logdet, int* info, bool inverse,
                   hipStream_t stream) {
  if (rocsolver_dpotrf(h, rocblas_fill_lower, n, A, lda, info) != rocblas_status_success) {
    set_error("rocsolver_dpotrf failed (n=%d)", n);
    return GPL_EHIP;
  }
  hipLaunchKernelGGL(diag_log_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, A, lda, logd);
  GPL_LAUNCH_CHECK();
  if (logdet) {
    hipLaunchKernelGGL(logdet_fold_kernel, dim3(1), dim3(64), 0, stream, n, logd, logdet);
    GPL_LAUNCH_CHECK();
  }
  if (inverse && rocsolver_dpotri(h, rocblas_fill_lower, n, A, lda, info) != rocblas_status_success) {
    set_error("rocsolver_dpotri failed (n=%d)", n);
    return GPL_EHIP;
  }
  return GPL_OK;
}

// One row of B per thread: x R^T = b, i.e. x_v = (b_v - sum_{w<v} x_w R[v][w]) / R[v][v].
// R is read from LDS at the same address by every lane (broadcast).
constexpr int kTri = 64;
__global__ __launch_bounds__(256) void trsm_rows64_kernel(int m, const double* __restrict__ R, double* B, int ldb) {
  __shared__ double Rl[kTri][kTri];  // Rl[v][w] = R[v][w]
  __shared__ double idg[kTri];
  for (int e = threadIdx.x; e < kTri * kTri; e += blockDim.x) {
    const int w = e / kTri, v = e - w * kTri;  // column-major: element (v, w) at w * 64 + v
    Rl[v][w] = R[e];
  }
  __syncthreads();
  if (threadIdx.x < kTri) idg[threadIdx.x] = 1.0 / Rl[threadIdx.x][threadIdx.x];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double x[kTri];
#pragma unroll
  for (int v = 0; v < kTri; ++v) x[v] = B[(size_t)v * ldb + i];
#pragma unroll
  for (int v = 0; v < kTri; ++v) {
    double acc = x[v];
#pragma unroll
    for (int w = 0; w < v; ++w) acc = fma(-x[w], Rl[v][w], acc);
    x[v] = acc * idg[v];
  }
#pragma unroll
  for (int v = 0; v < kTri; ++v) B[(size_t)v * ldb + i] = x[v];
}

int trsm_rows64(int m, const double* R, double* B, int ldb, hipStream_t stream) {
  if (m <= 0) return GPL_OK;
  hipLaunchKernelGGL(trsm_rows64_kernel, dim3(cdiv(m, 256)), dim3(256), 0, stream, m, R, B, ldb);
  GPL_LAUNCH_CHECK();
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
