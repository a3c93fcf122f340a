// Image grid (fine sub-pixel centres, pixel index map) and ray tracing through
// an SPLE lens with external shear (Sec. 2.1 lens equation; Sec. 2.2 elliptical
// coordinates, eq. "dispsple" and the shear deflection), plus its adjoint.
//
// The SPLE deflection is evaluated directly: e^{i varphi} = (R_x + i R_y)/R
// needs no trigonometry, 2F1(1, b; c; z) is summed by Horner's rule over a
// number of series terms fixed on the host from |z| = (1-q)/(1+q), and the
// lens-frame deflection is rotated back by -phi. One thread per fine point;
// the grid coordinates are generated in registers, never read from memory.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "dual.hpp"
#include "internal.hpp"

namespace gpl {

struct GridF {
  int n, ss, M;
  float h, x0, y0;  // x of fine column 0: cx - (M-1)/2 h
  float cx, cy;
};

static GridF make_grid(const gpl_grid* g) {
  GridF r;
  r.n = g->n;
  r.ss = g->ss;
  r.M = g->n * g->ss;
  r.h = (float)(g->pix_scale / g->ss);
  r.cx = (float)g->cx;
  r.cy = (float)g->cy;
  r.x0 = 0.f;
  r.y0 = 0.f;
  return r;
}

__device__ inline void fine_xy(const GridF& g, int j, float& x, float& y, int& pix) {
  const int fy = j / g.M, fx = j - fy * g.M;
  const float half = 0.5f * (float)(g.M - 1);
  x = g.cx + ((float)fx - half) * g.h;
  y = g.cy + ((float)fy - half) * g.h;
  pix = (fy / g.ss) * g.n + fx / g.ss;
}

static int check_grid(const gpl_grid* g) {
  GPL_REQUIRE(g != nullptr, "grid is NULL");
  GPL_REQUIRE(g->n >= 1 && g->ss >= 1, "grid n=%d ss=%d must be >= 1", g->n, g->ss);
  GPL_REQUIRE((long long)g->n * g->ss * g->n * g->ss < (1LL << 30), "grid too large");
  GPL_REQUIRE(g->pix_scale > 0 && std::isfinite(g->pix_scale), "pix_scale must be > 0");
  GPL_REQUIRE(std::isfinite(g->cx) && std::isfinite(g->cy), "grid centre must be finite");
  return GPL_OK;
}

static int check_lens(const gpl_lens* L) {
  GPL_REQUIRE(L != nullptr, "lens is NULL");
  GPL_REQUIRE(L->theta_E > 0 && std::isfinite(L->theta_E), "theta_E must be > 0");
  GPL_REQUIRE(L->q >= 0.02 && L->q <= 1.0, "q=%g must be in [0.02, 1]", L->q);
  GPL_REQUIRE(L->slope > 1.0 && L->slope < 3.0, "slope=%g must be in (1, 3)", L->slope);
  GPL_REQUIRE(std::isfinite(L->phi) && std::isfinite(L->x0) && std::isfinite(L->y0) && std::isfinite(L->gamma1) &&
                  std::isfinite(L->gamma2),
              "lens parameters must be finite");
  return GPL_OK;
}

// Series length: |t_k| <= |z|^k (the ratio (b+k)/(c+k) < 1 for slope < 3), so the
// tail after K terms is below |z|^K / (1-|z|); K makes it < 2^-27.
static int series_terms(double q) {
  const double z = (1.0 - q) / (1.0 + q);
  if (z < 1e-9) return 1;
  int K = (int)std::ceil(std::log(std::ldexp(1.0, -27) * (1.0 - z)) / std::log(z)) + 1;
  return K < 1 ? 1 : (K > 512 ? 512 : K);
}

template <class T>
struct LensCore {
  T cphi, sphi, sq, isq, pref, log2te, gm2, zmag, b, c, x0, y0;
};

// SPLE deflection at image-plane point (xix, xiy), sky frame.
template <class T>
__device__ inline void sple_deflect(float xix, float xiy, const LensCore<T>& L, int nterms, T& ax, T& ay) {
  const T dx = xix - L.x0, dy = xiy - L.y0;
  const T xp = L.cphi * dx + L.sphi * dy;
  const T yp = L.cphi * dy - L.sphi * dx;
  const T Rx = L.sq * xp, Ry = L.isq * yp;
  const T R2 = Rx * Rx + Ry * Ry;
  T R, ex, ey;
  if (value_of(R2) < 1e-18f) {  // R floor 1e-9 arcsec; varphi = 0 by convention
    R = T(1e-9f);
    ex = T(1.f);
    ey = T(0.f);
  } else {
    R = dsqrt(R2);
    const T iR = T(1.f) / R;
    ex = Rx * iR;
    ey = Ry * iR;
  }
  // z = -(1-q)/(1+q) e^{2 i varphi}
  const T zx = -(L.zmag * (ex * ex - ey * ey));
  const T zy = -(L.zmag * (2.f * (ex * ey)));
  // 2F1(1, b; c; z) = 1 + r_0 z (1 + r_1 z (1 + ...)), r_k = (b+k)/(c+k)
  T fx(1.f), fy(0.f);
  for (int k = nterms - 1; k >= 0; --k) {
    const T rk = (L.b + (float)k) / (L.c + (float)k);
    const T wx = rk * zx, wy = rk * zy;
    const T nx = 1.f + (wx * fx - wy * fy);
    const T ny = wx * fy + wy * fx;
    fx = nx;
    fy = ny;
  }
  // |alpha'| prefactor: theta_E 2 sqrt(q)/(1+q) (theta_E/R)^(slope-2)
  const T mag = L.pref * dexp2(L.gm2 * (L.log2te - dlog2(R)));
  const T apx = mag * (fx * ex - fy * ey);
  const T apy = mag * (fx * ey + fy * ex);
  ax = L.cphi * apx - L.sphi * apy;
  ay = L.sphi * apx + L.cphi * apy;
}

__global__ void grid_map_kernel(GridF g, int N, float* xi_x, float* xi_y, int* pix) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float x, y;
  int p;
  fine_xy(g, j, x, y, p);
  if (xi_x) xi_x[j] = x;
  if (xi_y) xi_y[j] = y;
  if (pix) pix[j] = p;
}

__device__ inline void trace_point(const GridF& g, int j, const LensCore<float>& L, float g1, float g2, int nterms,
                                   float* px, float* py) {
  float x, y;
  int p;
  fine_xy(g, j, x, y, p);
  float ax, ay;
  sple_deflect<float>(x, y, L, nterms, ax, ay);
  const float sx = g1 * x + g2 * y, sy = g2 * x - g1 * y;
  px[j] = x - ax - sx;
  py[j] = y - ay - sy;
}

__global__ void raytrace_kernel(GridF g, int N, LensCore<float> L, float g1, float g2, int nterms, float* px,
                                float* py) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  trace_point(g, j, L, g1, g2, nterms, px, py);
}

// Lens parameters held in device memory (8 doubles in gpl_lens order), as a
// sampled lens of the variational step keeps them: every thread derives the
// constants itself. Parameters outside the lens model's range give non-finite
// points, never an unbounded loop (the series length is capped).
__device__ inline gpl_lens lens_from(const double* p) {
  gpl_lens L;
  L.theta_E = p[0];
  L.q = p[1];
  L.phi = p[2];
  L.slope = p[3];
  L.x0 = p[4];
  L.y0 = p[5];
  L.gamma1 = p[6];
  L.gamma2 = p[7];
  return L;
}

__device__ inline int series_terms_dev(double q) {
  const double z = fabs((1.0 - q) / (1.0 + q));
  if (!(z < 1.0)) return 512;
  if (z < 1e-9) return 1;
  const int K = (int)ceil(log(ldexp(1.0, -27) * (1.0 - z)) / log(z)) + 1;
  return K < 1 ? 1 : (K > 512 ? 512 : K);
}

__device__ inline LensCore<float> lens_core_dev(const gpl_lens& L) {
  LensCore<float> c;
  c.cphi = (float)cos(L.phi);
  c.sphi = (float)sin(L.phi);
  c.sq = (float)sqrt(L.q);
  c.isq = (float)(1.0 / sqrt(L.q));
  c.pref = (float)(L.theta_E * 2.0 * sqrt(L.q) / (1.0 + L.q));
  c.log2te = (float)log2(L.theta_E);
  c.gm2 = (float)(L.slope - 2.0);
  c.zmag = (float)((1.0 - L.q) / (1.0 + L.q));
  c.b = (float)((L.slope - 1.0) / 2.0);
  c.c = (float)((5.0 - L.slope) / 2.0);
  c.x0 = (float)L.x0;
  c.y0 = (float)L.y0;
  return c;
}

__global__ void raytrace_dev_kernel(GridF g, int N, const double* __restrict__ lens, float* px, float* py) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const gpl_lens Lh = lens_from(lens);
  trace_point(g, j, lens_core_dev(Lh), (float)Lh.gamma1, (float)Lh.gamma2, series_terms_dev(Lh.q), px, py);
}

// Adjoint: per point, dp/dtheta for (theta_E, q, phi, slope, x0, y0) by forward-mode
// duals through sple_deflect; shear columns in closed form. Block partial sums in
// FP64 go to `partial[block][8]`.
__device__ inline void raytrace_backward_body(const GridF& g, int N, const gpl_lens& Lh, int nterms,
                                              const float* gpx, const float* gpy, double* partial) {
  using D6 = Dual<6>;
  __shared__ double red[4];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  if (j < N) {
    float x, y;
    int p;
    fine_xy(g, j, x, y, p);
    const D6 te = D6::var((float)Lh.theta_E, 0), q = D6::var((float)Lh.q, 1), phi = D6::var((float)Lh.phi, 2),
             sl = D6::var((float)Lh.slope, 3), x0 = D6::var((float)Lh.x0, 4), y0 = D6::var((float)Lh.y0, 5);
    LensCore<D6> L;
    L.cphi = dcos(phi);
    L.sphi = dsin(phi);
    L.sq = dsqrt(q);
    L.isq = D6(1.f) / L.sq;
    L.pref = te * (2.f * L.sq) / (1.f + q);
    L.log2te = dlog2(te);
    L.gm2 = sl - 2.f;
    L.zmag = (1.f - q) / (1.f + q);
    L.b = (sl - 1.f) * 0.5f;
    L.c = (5.f - sl) * 0.5f;
    L.x0 = x0;
    L.y0 = y0;
    D6 ax, ay;
    sple_deflect<D6>(x, y, L, nterms, ax, ay);
    const float gx = gpx[j], gy = gpy[j];
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = -(double)(gx * ax.d[k] + gy * ay.d[k]);
    acc[6] = (double)(-gx * x + gy * y);  // dp/dgamma1 = (-x, y)
    acc[7] = (double)(-gx * y - gy * x);  // dp/dgamma2 = (-y, -x)
  }
  for (int k = 0; k < 8; ++k) {
    const double s = block_sum_double(acc[k], red);
    if (threadIdx.x == 0) partial[blockIdx.x * 8 + k] = s;
  }
}

__global__ __launch_bounds__(256) void raytrace_backward_kernel(GridF g, int N, gpl_lens Lh, int nterms,
                                                                const float* gpx, const float* gpy,
                                                                double* partial) {
  raytrace_backward_body(g, N, Lh, nterms, gpx, gpy, partial);
}

__global__ __launch_bounds__(256) void raytrace_backward_dev_kernel(GridF g, int N, const double* __restrict__ lens,
                                                                    const float* gpx, const float* gpy,
                                                                    double* partial) {
  const gpl_lens Lh = lens_from(lens);
  raytrace_backward_body(g, N, Lh, series_terms_dev(Lh.q), gpx, gpy, partial);
}

__global__ void sum_partials_kernel(const double* partial, int nblocks, int width, double* out) {
  const int k = threadIdx.x;
  if (k >= width) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b * width + k];
  out[k] = s;
}

static LensCore<float> lens_core_float(const gpl_lens* L) {
  LensCore<float> c;
  c.cphi = (float)std::cos(L->phi);
  c.sphi = (float)std::sin(L->phi);
  c.sq = (float)std::sqrt(L->q);
  c.isq = (float)(1.0 / std::sqrt(L->q));
  c.pref = (float)(L->theta_E * 2.0 * std::sqrt(L->q) / (1.0 + L->q));
  c.log2te = (float)std::log2(L->theta_E);
  c.gm2 = (float)(L->slope - 2.0);
  c.zmag = (float)((1.0 - L->q) / (1.0 + L->q));
  c.b = (float)((L->slope - 1.0) / 2.0);
  c.c = (float)((5.0 - L->slope) / 2.0);
  c.x0 = (float)L->x0;
  c.y0 = (float)L->y0;
  return c;
}

// Scratch of the allocation-free adjoint: 8 partial sums per 256-point block,
// for up to kNoAllocMaxBlocks blocks (grids of up to 4,194,304 fine points),
// 1 MiB held by each device the library runs on until the process ends. Host
// code uses it only through the device address recorded per device below.
constexpr int kNoAllocMaxBlocks = 16384;
static __device__ __align__(256) double scratch[kNoAllocMaxBlocks * 8];

static std::mutex g_scratch_mutex;
static double* g_scratch_ptr[64] = {};

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
static int scratch_address(double** out) {
  int dev = 0;
  GPL_HIP(hipGetDevice(&dev));
  GPL_REQUIRE(dev >= 0 && dev < 64, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    GPL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    GPL_REQUIRE(ptr != nullptr, "no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return GPL_OK;
}

size_t raytrace_dev_backward_scratch(int N) { return align_up(sizeof(double) * 8 * (size_t)cdiv(N, 256)); }

int raytrace_dev_launch(const gpl_grid* grid, const double* lens, float* px, float* py, hipStream_t stream) {
  GPL_TRY(check_grid(grid));
  const GridF g = make_grid(grid);
  const int N = g.M * g.M;
  hipLaunchKernelGGL(raytrace_dev_kernel, dim3(cdiv(N, 256)), dim3(256), 0, stream, g, N, lens, px, py);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int raytrace_dev_backward_launch(const gpl_grid* grid, const double* lens, const float* gpx, const float* gpy,
                                 double* g_lens, double* scratch_partial, hipStream_t stream) {
  GPL_TRY(check_grid(grid));
  const GridF g = make_grid(grid);
  const int N = g.M * g.M, nb = cdiv(N, 256);
  hipLaunchKernelGGL(raytrace_backward_dev_kernel, dim3(nb), dim3(256), 0, stream, g, N, lens, gpx, gpy,
                     scratch_partial);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, stream, scratch_partial, nb, 8, g_lens);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" int gpl_grid_map(const gpl_grid* grid, float* xi_x, float* xi_y, int* pixel_of_fine, hipStream_t stream) {
  GPL_TRY(check_grid(grid));
  const GridF g = make_grid(grid);
  const int N = g.M * g.M;
  hipLaunchKernelGGL(grid_map_kernel, dim3(cdiv(N, 256)), dim3(256), 0, stream, g, N, xi_x, xi_y, pixel_of_fine);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" int gpl_lens_raytrace(const gpl_grid* grid, const gpl_lens* lens, float* px, float* py,
                                 hipStream_t stream) {
  GPL_TRY(check_grid(grid));
  GPL_TRY(check_lens(lens));
  GPL_REQUIRE(px != nullptr && py != nullptr, "px/py are NULL");
  const GridF g = make_grid(grid);
  const int N = g.M * g.M;
  hipLaunchKernelGGL(raytrace_kernel, dim3(cdiv(N, 256)), dim3(256), 0, stream, g, N, lens_core_float(lens),
                     (float)lens->gamma1, (float)lens->gamma2, series_terms(lens->q), px, py);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" size_t gpl_lens_raytrace_backward_workspace(const gpl_grid* grid) {
  if (check_grid(grid) != GPL_OK) return 0;
  const int N = grid->n * grid->ss * grid->n * grid->ss;
  return align_up(sizeof(double) * 8 * (size_t)cdiv(N, 256));
}

extern "C" int gpl_lens_raytrace_backward(const gpl_grid* grid, const gpl_lens* lens, const float* gpx,
                                          const float* gpy, double* g_lens, void* ws, size_t ws_bytes,
                                          hipStream_t stream) {
  GPL_TRY(check_grid(grid));
  GPL_TRY(check_lens(lens));
  GPL_REQUIRE(gpx && gpy && g_lens, "gpx/gpy/g_lens are NULL");
  GPL_TRY(check_ws(ws, ws_bytes, gpl_lens_raytrace_backward_workspace(grid)));
  const GridF g = make_grid(grid);
  const int N = g.M * g.M, nb = cdiv(N, 256);
  double* partial = static_cast<double*>(ws);
  hipLaunchKernelGGL(raytrace_backward_kernel, dim3(nb), dim3(256), 0, stream, g, N, *lens, series_terms(lens->q),
                     gpx, gpy, partial);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, stream, partial, nb, 8, g_lens);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" int gpl_lens_raytrace_backward_noalloc(const gpl_grid* grid, const gpl_lens* lens, const float* gpx,
                                                  const float* gpy, double* g_lens, hipStream_t stream) {
  GPL_TRY(check_grid(grid));
  GPL_TRY(check_lens(lens));
  GPL_REQUIRE(gpx && gpy && g_lens, "gpx/gpy/g_lens are NULL");
  const GridF g = make_grid(grid);
  const int N = g.M * g.M, nb = cdiv(N, 256);
  GPL_REQUIRE(nb <= kNoAllocMaxBlocks, "grid of %d fine points exceeds the %d the static scratch holds", N,
              kNoAllocMaxBlocks * 256);
  double* partial = nullptr;
  GPL_TRY(scratch_address(&partial));
  // every block writes its 8 partial sums before they are read: nothing to clear
  hipLaunchKernelGGL(raytrace_backward_kernel, dim3(nb), dim3(256), 0, stream, g, N, *lens, series_terms(lens->q),
                     gpx, gpy, partial);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, stream, partial, nb, 8, g_lens);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
