// Stochastic Lanczos quadrature of ln|A| from the CG coefficients (the
// stochastic log-determinant discussed in Sec. 3.3 for eq. "gp-mll").
//
// For probe j the k x k tridiagonal T implied by CG, T_kk = 1/a_k + b_{k-1}/a_{k-1},
// T_{k,k+1} = sqrt(b_k)/a_k, gives z^T ln(A) z ~= |z|^2 e_1^T ln(T) e_1 (Gauss
// quadrature on the Ritz values). Instead of diagonalising T, the quadratic form
// is evaluated from the integral representation of the logarithm,
//   ln x = int_R e^s [ 1/(1 + e^s) - 1/(x + e^s) ] ds,
// so e_1^T ln(T) e_1 = int e^s [ 1/(1 + e^s) - e_1^T (T + e^s I)^{-1} e_1 ] ds.
// The integrand is analytic in the strip |Im s| < pi (poles at s = ln x + i pi),
// so the trapezoidal rule with step h converges like exp(-2 pi^2 / h); nodes run
// from ln(x_hi) - 75 to ln(x_hi) + 38 (x_hi a Gershgorin bound), where the
// integrand is below 1e-16. Each resolvent element (T + tI)^{-1}_{11} is a
// continued fraction evaluated from the bottom of T (the pivots of an LDL^T
// factorisation, all positive for t >= 0 when T is positive definite).
// One wave per probe: the coefficients sit in LDS, lanes take the nodes, a
// fixed-order reduction sums them (FP64 throughout).
#include <cmath>

#include "common.hpp"

namespace gpl {

constexpr int kSlqMaxSteps = 4096;       // LDS capacity per probe (doubles x 2)
constexpr double kSlqStep = 0.4;         // trapezoid step in s = ln t
constexpr double kSlqLo = 75.0, kSlqHi = 38.0;

__global__ __launch_bounds__(64) void slq_probe_kernel(int nprobe, int n_lanczos, const double* __restrict__ ab,
                                                       const int* __restrict__ iters,
                                                       const double* __restrict__ bnorm2, double* contrib) {
  __shared__ double diag[kSlqMaxSteps];
  __shared__ double off2[kSlqMaxSteps];
  __shared__ double s_hi;
  __shared__ int s_ok;
  const int j = blockIdx.x, lane = threadIdx.x;
  const int m = min(iters[j], n_lanczos);
  if (m <= 0) {
    if (lane == 0) contrib[j] = 0.0;
    return;
  }
  const double* a = ab + (size_t)j * n_lanczos * 2;
  for (int k = lane; k < m; k += 64) {
    const double ak = a[2 * k], bk = a[2 * k + 1];
    double dk = 1.0 / ak;
    if (k > 0) dk += a[2 * (k - 1) + 1] / a[2 * (k - 1)];
    diag[k] = dk;
    off2[k] = (k + 1 < m) ? bk / (ak * ak) : 0.0;  // (sqrt(b_k)/a_k)^2
  }
  __syncthreads();
  if (lane == 0) {
    // positive definiteness (all pivots of T from the bottom positive) and a
    // Gershgorin upper bound of the spectrum
    double g = diag[m - 1];
    int ok = g > 0.0;
    double hi = diag[m - 1] + (m > 1 ? sqrt(off2[m - 2]) : 0.0);
    for (int k = m - 2; k >= 0; --k) {
      g = diag[k] - off2[k] / g;
      ok &= g > 0.0;
      const double r = sqrt(off2[k]) + (k > 0 ? sqrt(off2[k - 1]) : 0.0);
      hi = fmax(hi, diag[k] + r);
    }
    s_ok = ok && isfinite(g);
    s_hi = hi;
  }
  __syncthreads();
  if (!s_ok) {
    if (lane == 0) contrib[j] = __builtin_nan("");
    return;
  }
  const double s_lo = log(s_hi) - kSlqLo;
  const int nodes = (int)((kSlqLo + kSlqHi) / kSlqStep) + 1;
  double acc = 0.0;
  for (int q = lane; q < nodes; q += 64) {
    const double t = exp(s_lo + q * kSlqStep);
    double g = diag[m - 1] + t;
    for (int k = m - 2; k >= 0; --k) g = (diag[k] + t) - off2[k] / g;
    acc += t * (1.0 / (1.0 + t) - 1.0 / g);
  }
  acc = warp_sum(acc);
  if (lane == 0) contrib[j] = bnorm2[j] * kSlqStep * acc;
}

__global__ void slq_sum_kernel(int nprobe, double scale, const double* offset, const double* contrib, double* logdet,
                               double* stderr_out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int j = 0; j < nprobe; ++j) s += contrib[j];
  const double mean = s / nprobe;
  double v = 0.0;
  for (int j = 0; j < nprobe; ++j) v += (contrib[j] - mean) * (contrib[j] - mean);
  *logdet = scale * s + (offset ? *offset : 0.0);
  // sample standard deviation of the contributions, scaled like the estimate
  *stderr_out = nprobe > 1 ? scale * sqrt(v / (nprobe - 1)) * sqrt((double)nprobe) : NAN;
}

}  // namespace gpl

using namespace gpl;

extern "C" size_t gpl_lanczos_logdet_workspace(int nprobe, int n_lanczos) {
  (void)nprobe;
  (void)n_lanczos;
  return 0;  // coefficients are staged in LDS
}

extern "C" int gpl_lanczos_logdet(int nprobe, int n_lanczos, const double* lanczos_ab, const int* iters,
                                  const double* bnorm2, double scale, const double* offset, double* contrib,
                                  double* logdet, double* stderr_out, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
  GPL_REQUIRE(nprobe >= 1 && n_lanczos >= 1, "nprobe=%d n_lanczos=%d must be >= 1", nprobe, n_lanczos);
  GPL_REQUIRE(lanczos_ab && iters && bnorm2 && contrib && logdet && stderr_out, "NULL argument");
  GPL_REQUIRE(std::isfinite(scale), "scale must be finite");
  GPL_REQUIRE(n_lanczos <= kSlqMaxSteps, "n_lanczos=%d exceeds %d", n_lanczos, kSlqMaxSteps);
  (void)ws;
  (void)ws_bytes;
  hipLaunchKernelGGL(slq_probe_kernel, dim3(nprobe), dim3(64), 0, stream, nprobe, n_lanczos, lanczos_ab, iters,
                     bnorm2, contrib);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(slq_sum_kernel, dim3(1), dim3(64), 0, stream, nprobe, scale, offset, contrib, logdet,
                     stderr_out);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
