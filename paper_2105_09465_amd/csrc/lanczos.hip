// Stochastic Lanczos quadrature of ln|A| from the CG coefficients (the
// stochastic log-determinant discussed in Sec. 3.3 for eq. "gp-mll").
//
// For probe j the k x k tridiagonal T implied by CG, T_kk = 1/a_k + b_{k-1}/a_{k-1},
// T_{k,k+1} = sqrt(b_k)/a_k, is diagonalised in FP64 by implicit symmetric QR
// steps with a Wilkinson shift (bulge chasing with Givens rotations), keeping
// only the first row of the accumulated rotations: z^T ln(A) z is approximated
// by |z|^2 sum_i q_i^2 ln(theta_i) (Gauss quadrature on the Ritz values theta_i
// with weights q_i^2). One thread per probe; the per-probe arrays live in the
// workspace. A second kernel sums the contributions in a fixed order.
#include <cmath>

#include "common.hpp"

namespace gpl {

// Eigenvalues (left in d) and first eigenvector components (q) of the
// symmetric tridiagonal (d[0..m-1], e[0..m-2]).
__device__ void tridiag_eig_first(int m, double* d, double* e, double* q) {
  for (int i = 0; i < m; ++i) q[i] = (i == 0) ? 1.0 : 0.0;
  int hi = m - 1;
  int sweeps = 0;
  const double eps = 2.220446049250313e-16;
  while (hi > 0 && sweeps < 50 * m) {
    // deflate converged eigenvalues at the bottom
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    // Wilkinson shift from the trailing 2x2 block
    const double t = 0.5 * (d[hi - 1] - d[hi]);
    const double bb = e[hi - 1] * e[hi - 1];
    const double sgn = t >= 0.0 ? 1.0 : -1.0;
    const double mu = d[hi] - bb / (t + sgn * sqrt(t * t + bb));
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = hypot(x, z);
      const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? z / r : 0.0;
      if (k > lo) e[k - 1] = r;
      const double ak = d[k], ak1 = d[k + 1], bk = e[k];
      d[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      d[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      e[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        x = e[k];
        z = s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      const double qk = q[k], qk1 = q[k + 1];
      q[k] = c * qk + s * qk1;
      q[k + 1] = -s * qk + c * qk1;
    }
    ++sweeps;
  }
}

__global__ void slq_probe_kernel(int nprobe, int n_lanczos, const double* __restrict__ ab, const int* __restrict__ iters,
                                 const double* __restrict__ bnorm2, double* contrib, double* scratch) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nprobe) return;
  const int m = min(iters[j], n_lanczos);
  double* d = scratch + (size_t)j * 3 * n_lanczos;
  double* e = d + n_lanczos;
  double* q = e + n_lanczos;
  if (m <= 0) {
    contrib[j] = 0.0;
    return;
  }
  const double* a = ab + (size_t)j * n_lanczos * 2;
  for (int k = 0; k < m; ++k) {
    const double ak = a[2 * k], bk = a[2 * k + 1];
    d[k] = 1.0 / ak;
    if (k > 0) d[k] += a[2 * (k - 1) + 1] / a[2 * (k - 1)];
    if (k + 1 < m) e[k] = sqrt(bk) / ak;
  }
  if (m > 1) e[m - 1] = 0.0;
  tridiag_eig_first(m, d, e, q);
  double s = 0.0;
  for (int k = 0; k < m; ++k) s += q[k] * q[k] * log(d[k]);  // log of a non-positive Ritz value gives NaN
  contrib[j] = bnorm2[j] * s;
}

__global__ void slq_sum_kernel(int nprobe, double scale, const double* contrib, double* logdet, double* stderr_out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int j = 0; j < nprobe; ++j) s += contrib[j];
  const double mean = s / nprobe;
  double v = 0.0;
  for (int j = 0; j < nprobe; ++j) v += (contrib[j] - mean) * (contrib[j] - mean);
  *logdet = scale * s;
  // sample standard deviation of the contributions, scaled like the estimate
  *stderr_out = nprobe > 1 ? scale * sqrt(v / (nprobe - 1)) * sqrt((double)nprobe) : NAN;
}

}  // namespace gpl

using namespace gpl;

extern "C" size_t gpl_lanczos_logdet_workspace(int nprobe, int n_lanczos) {
  if (nprobe <= 0 || n_lanczos <= 0) return 0;
  return align_up(sizeof(double) * 3 * (size_t)n_lanczos * nprobe);
}

extern "C" int gpl_lanczos_logdet(int nprobe, int n_lanczos, const double* lanczos_ab, const int* iters,
                                  const double* bnorm2, double scale, double* contrib, double* logdet,
                                  double* stderr_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  GPL_REQUIRE(nprobe >= 1 && n_lanczos >= 1, "nprobe=%d n_lanczos=%d must be >= 1", nprobe, n_lanczos);
  GPL_REQUIRE(lanczos_ab && iters && bnorm2 && contrib && logdet && stderr_out, "NULL argument");
  GPL_REQUIRE(std::isfinite(scale), "scale must be finite");
  GPL_TRY(check_ws(ws, ws_bytes, gpl_lanczos_logdet_workspace(nprobe, n_lanczos)));
  hipLaunchKernelGGL(slq_probe_kernel, dim3(cdiv(nprobe, 64)), dim3(64), 0, stream, nprobe, n_lanczos, lanczos_ab,
                     iters, bnorm2, contrib, static_cast<double*>(ws));
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(slq_sum_kernel, dim3(1), dim3(64), 0, stream, nprobe, scale, contrib, logdet, stderr_out);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
