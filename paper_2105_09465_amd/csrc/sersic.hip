// Sersic mean function of the GP source (mean function footnote of Sec. 3.1)
// and its adjoint. mu = I_e exp(-b_n ((r/R_e)^(1/n) - 1)), r = |p - p_s|.
#include <cmath>

#include "common.hpp"

namespace gpl {

struct SersicF {
  float I_e, inv_Re, inv_n, bn_log2e, bn, xs, ys;
};

static SersicF make_sersic(const gpl_source* s) {
  SersicF f;
  f.I_e = (float)s->I_e;
  f.inv_Re = (float)(1.0 / s->R_e);
  f.inv_n = (float)(1.0 / s->n_sersic);
  f.bn_log2e = (float)(s->b_n * 1.4426950408889634);
  f.bn = (float)s->b_n;
  f.xs = (float)s->xs;
  f.ys = (float)s->ys;
  return f;
}

static int check_source(const gpl_source* s) {
  GPL_REQUIRE(s != nullptr, "source is NULL");
  GPL_REQUIRE(s->R_e > 0 && s->n_sersic > 0 && s->b_n > 0, "Sersic R_e, n, b_n must be > 0");
  GPL_REQUIRE(std::isfinite(s->I_e) && std::isfinite(s->xs) && std::isfinite(s->ys), "Sersic parameters must be finite");
  return GPL_OK;
}

// (r/R_e)^(1/n) via exp2(log2(.)/n); r = 0 gives exp2(-inf) = 0.
__device__ inline float sersic_shape(const SersicF& S, float dx, float dy, float& t) {
  const float r = sqrtf(dx * dx + dy * dy);
  t = exp2f(log2f(r * S.inv_Re) * S.inv_n);
  return S.I_e * exp2f(S.bn_log2e * (1.f - t));
}

__global__ void sersic_kernel(SersicF S, int n, const float* px, const float* py, float* mu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float t;
  mu[i] = sersic_shape(S, px[i] - S.xs, py[i] - S.ys, t);
}

__global__ __launch_bounds__(256) void sersic_backward_kernel(SersicF S, int n, const float* px, const float* py,
                                                              const float* gmu, float* gpx, float* gpy,
                                                              double* partial) {
  __shared__ double red[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double ax = 0.0, ay = 0.0;
  if (i < n) {
    const float dx = px[i] - S.xs, dy = py[i] - S.ys;
    float t;
    const float m = sersic_shape(S, dx, dy, t);
    const float r2 = dx * dx + dy * dy;
    // dmu/dp = -mu b_n/n (r/R_e)^(1/n) (dx, dy)/r^2; zero at r = 0 by convention
    const float f = r2 > 0.f ? -m * S.bn * S.inv_n * t / r2 : 0.f;
    const float gx = gmu[i] * f * dx, gy = gmu[i] * f * dy;
    gpx[i] += gx;
    gpy[i] += gy;
    ax = -(double)gx;  // d/dxs = -d/dpx
    ay = -(double)gy;
  }
  const double sx = block_sum_double(ax, red);
  if (threadIdx.x == 0) partial[blockIdx.x * 2 + 0] = sx;
  const double sy = block_sum_double(ay, red);
  if (threadIdx.x == 0) partial[blockIdx.x * 2 + 1] = sy;
}

__global__ void sum_partials2_kernel(const double* partial, int nblocks, double* out) {
  const int k = threadIdx.x;
  if (k >= 2) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b * 2 + k];
  out[k] = s;
}

}  // namespace gpl

using namespace gpl;

extern "C" int gpl_sersic_eval(const gpl_source* src, int n, const float* px, const float* py, float* mu,
                               hipStream_t stream) {
  GPL_TRY(check_source(src));
  GPL_REQUIRE(n >= 0, "n=%d must be >= 0", n);
  if (n == 0) return GPL_OK;
  GPL_REQUIRE(px && py && mu, "px/py/mu are NULL");
  hipLaunchKernelGGL(sersic_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, make_sersic(src), n, px, py, mu);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" size_t gpl_sersic_backward_workspace(int n) {
  return n <= 0 ? 0 : align_up(sizeof(double) * 2 * (size_t)cdiv(n, 256));
}

extern "C" int gpl_sersic_backward(const gpl_source* src, int n, const float* px, const float* py, const float* gmu,
                                   float* gpx, float* gpy, double* g_src, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
  GPL_TRY(check_source(src));
  GPL_REQUIRE(n >= 1, "n=%d must be >= 1", n);
  GPL_REQUIRE(px && py && gmu && gpx && gpy && g_src, "NULL argument");
  GPL_TRY(check_ws(ws, ws_bytes, gpl_sersic_backward_workspace(n)));
  const int nb = cdiv(n, 256);
  double* partial = static_cast<double*>(ws);
  hipLaunchKernelGGL(sersic_backward_kernel, dim3(nb), dim3(256), 0, stream, make_sersic(src), n, px, py, gmu, gpx,
                     gpy, partial);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_partials2_kernel, dim3(1), dim3(64), 0, stream, partial, nb, g_src);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
