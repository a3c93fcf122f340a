// Error reporting, version, host-side helpers and the evidence scalars.
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace gpl {

static thread_local char g_last_error[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_last_error; }

// Regularised lower incomplete gamma P(a, x) from its power series
// e^{-x} x^a / Gamma(a+1) * sum_k x^k / ((a+1)...(a+k)).
static double inc_gamma_p(double a, double x) {
  if (x <= 0) return 0.0;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 10000; ++k) {
    term *= x / (a + k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return std::exp(a * std::log(x) - x - std::lgamma(a + 1.0)) * sum;
}

// Evidence scalars: quad = r.u, ln p and the App. D.1 loss.
__global__ void evidence_scalars_kernel(int n_pix, int n_points, const float* r, const float* u, const double* logdet,
                                        double amp, double sigma, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n_pix; i += blockDim.x) s += (double)r[i] * (double)u[i];
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) {
    const double ln2pi = 1.8378770664093454835606594728112;
    out[0] = s;
    out[1] = -0.5 * (s + *logdet + n_pix * ln2pi);
    out[2] = s + n_points * log(amp * amp + sigma * sigma);
  }
}

// out[c] = sum_i X[c][i] * Y[c][i] in FP64, one workgroup per column.
__global__ __launch_bounds__(256) void block_dot_kernel(int n, const float* __restrict__ X, int ldx,
                                                        const float* __restrict__ Y, int ldy, double* out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += (double)X[(size_t)c * ldx + i] * (double)Y[(size_t)c * ldy + i];
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) out[c] = s;
}

// out[c] = prior - sum_i W[c][i] X[c][i] (FP64, one workgroup per column).
__global__ __launch_bounds__(256) void posterior_variance_kernel(int n, const float* __restrict__ W, int ldw,
                                                                 const float* __restrict__ X, int ldx, double prior,
                                                                 double* out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += (double)W[(size_t)c * ldw + i] * (double)X[(size_t)c * ldx + i];
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) out[c] = prior - s;
}

// Amplitude derivatives of ln p and of the App. D.1 loss. K is proportional to
// alpha^2, so alpha dA/dalpha = 2 B K B^T = 2 (A - sigma^2 I) and
//   alpha d ln p/d alpha = u^T B K B^T u - tr(A^{-1} B K B^T)
//                        = (quad - sigma^2 u.u) - (n - sigma^2 tr(A^{-1})),
// with tr(A^{-1}) and n = tr(I) estimated from the probes z_j and their solves
// x_j = A^{-1} z_j as scale * sum_j (|z_j|^2 - sigma^2 z_j.x_j);
//   d L_VI/d alpha = -2 (quad - sigma^2 u.u)/alpha + 2 N alpha/(alpha^2 + sigma^2).
// One workgroup; every dot product in FP64 in a fixed order.
__global__ __launch_bounds__(256) void amplitude_grad_kernel(int n_pix, int n_points, int nprobe,
                                                             const float* __restrict__ u, const float* __restrict__ Z,
                                                             int ldz, const float* __restrict__ X, int ldx,
                                                             const double* quad, double scale, double amp,
                                                             double sigma, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n_pix; i += blockDim.x) s += (double)u[i] * (double)u[i];
  const double uu = block_sum_double(s, red);
  double tr = 0.0;  // thread 0: scale * sum_j (|z_j|^2 - sigma^2 z_j.x_j)
  for (int j = 0; j < nprobe; ++j) {
    double zz = 0.0, zx = 0.0;
    for (int i = threadIdx.x; i < n_pix; i += blockDim.x) {
      const double z = Z[(size_t)j * ldz + i];
      zz += z * z;
      zx += z * (double)X[(size_t)j * ldx + i];
    }
    zz = block_sum_double(zz, red);
    zx = block_sum_double(zx, red);
    tr += zz - sigma * sigma * zx;
  }
  if (threadIdx.x == 0) {
    const double q = *quad - sigma * sigma * uu;  // u^T B K B^T u
    out[0] = (q - scale * tr) / amp;
    out[1] = -2.0 * q / amp + 2.0 * n_points * amp / (amp * amp + sigma * sigma);
  }
}

}  // namespace gpl

using namespace gpl;

extern "C" int gpl_evidence_amplitude_grad(int n_pix, int n_points, int nprobe, const float* u, const float* Z,
                                           int ldz, const float* X, int ldx, const double* quad, double scale,
                                           double amplitude, double noise_sigma, double* out, hipStream_t stream) {
  GPL_REQUIRE(n_pix >= 1 && n_points >= 1 && nprobe >= 0, "bad sizes");
  GPL_REQUIRE(u && quad && out, "NULL argument");
  GPL_REQUIRE(nprobe == 0 || (Z && X && ldz >= n_pix && ldx >= n_pix), "probe blocks NULL or ld < n_pix");
  GPL_REQUIRE(amplitude > 0 && std::isfinite(amplitude), "amplitude must be > 0");
  GPL_REQUIRE(noise_sigma >= 0 && std::isfinite(noise_sigma), "noise_sigma must be >= 0");
  hipLaunchKernelGGL(amplitude_grad_kernel, dim3(1), dim3(256), 0, stream, n_pix, n_points, nprobe, u, Z, ldz, X, ldx,
                     quad, scale, amplitude, noise_sigma, out);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" int gpl_block_dot(int n, int ncols, const float* X, int ldx, const float* Y, int ldy, double* out,
                             hipStream_t stream) {
  GPL_REQUIRE(n >= 0 && ncols >= 0, "negative size");
  if (ncols == 0) return GPL_OK;
  GPL_REQUIRE(X && Y && out, "NULL argument");
  GPL_REQUIRE(ldx >= n && ldy >= n, "ldx/ldy must be >= n");
  hipLaunchKernelGGL(block_dot_kernel, dim3(ncols), dim3(256), 0, stream, n, X, ldx, Y, ldy, out);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" int gpl_posterior_variance(int n, int ncols, const float* W, int ldw, const float* X, int ldx,
                                      double prior, double* out, hipStream_t stream) {
  GPL_REQUIRE(n >= 0 && ncols >= 0, "negative size");
  if (ncols == 0) return GPL_OK;
  GPL_REQUIRE(W && X && out, "NULL argument");
  GPL_REQUIRE(ldw >= n && ldx >= n, "ldw/ldx must be >= n");
  GPL_REQUIRE(std::isfinite(prior), "prior variance must be finite");
  hipLaunchKernelGGL(posterior_variance_kernel, dim3(ncols), dim3(256), 0, stream, n, W, ldw, X, ldx, prior, out);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" const char* gpl_strerror(int code) {
  switch (code) {
    case GPL_OK: return "ok";
    case GPL_EINVAL: return "invalid argument";
    case GPL_EWORKSPACE: return "workspace missing, misaligned or too small";
    case GPL_EHIP: return "HIP runtime error";
    case GPL_EUNSUPPORTED: return "unsupported precision or kind";
    default: return "unknown error";
  }
}

extern "C" const char* gpl_last_error(void) { return last_error(); }

extern "C" int gpl_version(void) { return 100; }

extern "C" double gpl_sersic_bn(double n) {
  if (!(n > 0) || !std::isfinite(n)) return NAN;
  const double a = 2.0 * n;
  double x = a - 1.0 / 3.0 > 0.05 ? a - 1.0 / 3.0 : 0.05;  // the median of Gamma(a, 1) is close to a - 1/3
  for (int it = 0; it < 100; ++it) {
    const double f = inc_gamma_p(a, x) - 0.5;
    const double fp = std::exp((a - 1.0) * std::log(x) - x - std::lgamma(a));  // density of Gamma(a, 1)
    double step = f / fp;
    double xn = x - step;
    if (xn <= 0) xn = 0.5 * x;
    if (std::fabs(xn - x) <= 1e-15 * x) {
      x = xn;
      break;
    }
    x = xn;
  }
  return x;
}

extern "C" int gpl_evidence_scalars(int n_pix, int n_points, const float* r, const float* u, const double* logdet,
                                    double amplitude, double noise_sigma, double* out, hipStream_t stream) {
  GPL_REQUIRE(n_pix >= 1 && n_points >= 1, "sizes must be >= 1");
  GPL_REQUIRE(r && u && logdet && out, "NULL argument");
  hipLaunchKernelGGL(evidence_scalars_kernel, dim3(1), dim3(256), 0, stream, n_pix, n_points, r, u, logdet, amplitude,
                     noise_sigma, out);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
