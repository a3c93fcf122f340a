// Gaussian products with per-point covariances: the pixel-shape (windowed)
// kernel of Sec. 3.2 (eq. "covariance"), the transmission matrix of Sec. 3.4
// (eq. "transmission") and its transpose, and the source reconstruction of
// Sec. 3.5 (eq. "gp-reconstruction"). All are sums
//   Y[i][c] = beta Y[i][c] + norm * wt_i * sum_j ws_j |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2) V[j][c],
//   d = t_i - s_j,  C_ij = Zt_i + Zs_j + base_var I  (2 x 2),
// over target points t and source points s, each optionally with a shape
// covariance Z (three floats: xx, xy, yy) and a weight w. One thread per target,
// 256 targets per workgroup; source tiles of 256 points and their right-hand
// side rows are staged in LDS; the exp tile is evaluated in FP32 on the fly and
// never stored. Dense over all pairs (every pair is evaluated).
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace gpl {

constexpr int kGTile = 256;  // sources per LDS tile = targets per workgroup
constexpr int kGCols = 8;    // right-hand-side columns per pass

__global__ __launch_bounds__(kGTile) void gauss_product_kernel(GSide T, GSide S, float base, float norm, int nc,
                                                               const float* __restrict__ V, int ldv, float* Y,
                                                               int ldy, float beta) {
  __shared__ float sx[kGTile], sy[kGTile], sxx[kGTile], sxy[kGTile], syy[kGTile], sw[kGTile];
  __shared__ float sv[kGCols][kGTile];
  const int i = blockIdx.x * kGTile + threadIdx.x;
  const bool live = i < T.n;
  const float xi = live ? T.x[i] : 0.f, yi = live ? T.y[i] : 0.f;
  const float txx = (live && T.z) ? T.z[i] : 0.f, txy = (live && T.z) ? T.z[T.n + i] : 0.f,
              tyy = (live && T.z) ? T.z[2 * T.n + i] : 0.f;
  float acc[kGCols];
#pragma unroll
  for (int c = 0; c < kGCols; ++c) acc[c] = 0.f;
  const float mh = -0.5f * 1.4426950408889634f;  // exp(-q/2) = exp2(mh q)
  for (int j0 = 0; j0 < S.n; j0 += kGTile) {
    __syncthreads();
    const int j = j0 + threadIdx.x;
    const bool sj = j < S.n;
    sx[threadIdx.x] = sj ? S.x[j] : 0.f;
    sy[threadIdx.x] = sj ? S.y[j] : 0.f;
    sxx[threadIdx.x] = (sj && S.z) ? S.z[j] : 0.f;
    sxy[threadIdx.x] = (sj && S.z) ? S.z[S.n + j] : 0.f;
    syy[threadIdx.x] = (sj && S.z) ? S.z[2 * S.n + j] : 0.f;
    sw[threadIdx.x] = sj ? (S.w ? S.w[j] : 1.f) : 0.f;
#pragma unroll
    for (int c = 0; c < kGCols; ++c) sv[c][threadIdx.x] = (sj && c < nc) ? V[(size_t)c * ldv + j] : 0.f;
    __syncthreads();
    const int cnt = min(kGTile, S.n - j0);
    for (int jj = 0; jj < cnt; ++jj) {
      const float cxx = txx + sxx[jj] + base, cxy = txy + sxy[jj], cyy = tyy + syy[jj] + base;
      const float det = fmaf(cxx, cyy, -cxy * cxy);
      const float dx = xi - sx[jj], dy = yi - sy[jj];
      const float q = fmaf(cyy * dx, dx, fmaf(-2.f * cxy * dx, dy, cxx * dy * dy)) / det;
      const float val = sw[jj] * rsqrtf(det) * exp2_fast(mh * q);
#pragma unroll
      for (int c = 0; c < kGCols; ++c) acc[c] = fmaf(val, sv[c][jj], acc[c]);
    }
  }
  if (!live) return;
  const float f = norm * (T.w ? T.w[i] : 1.f);
  for (int c = 0; c < nc; ++c) {
    float* y = Y + (size_t)c * ldy + i;
    *y = beta != 0.f ? f * acc[c] + beta * *y : f * acc[c];
  }
}

// Pixel shapes of the points of an M x M grid (row-major): a, b the half
// differences of the neighbouring projected centres along x and y (one-sided at
// the edges, footnote to eq. "window-kernel"), Z = (a a^T + b b^T) / (4 pi).
__global__ void pixel_shapes_kernel(int M, const float* __restrict__ px, const float* __restrict__ py, float* z) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = M * M;
  if (j >= N) return;
  const int fy = j / M, fx = j - fy * M;
  auto diff = [&](int lo, int hi, float h) -> float2 {  // (p[hi] - p[lo]) * h
    return make_float2((px[hi] - px[lo]) * h, (py[hi] - py[lo]) * h);
  };
  float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
  if (M > 1) {
    if (fx == 0) a = diff(j, j + 1, 1.f);
    else if (fx == M - 1) a = diff(j - 1, j, 1.f);
    else a = diff(j - 1, j + 1, 0.5f);
    if (fy == 0) b = diff(j, j + M, 1.f);
    else if (fy == M - 1) b = diff(j - M, j, 1.f);
    else b = diff(j - M, j + M, 0.5f);
  }
  const float f = (float)(1.0 / (4.0 * M_PI));
  z[j] = f * (a.x * a.x + b.x * b.x);
  z[N + j] = f * (a.x * a.y + b.x * b.y);
  z[2 * N + j] = f * (a.y * a.y + b.y * b.y);
}

// rho_i = k / (pi r_k^2), r_k the distance from point i to its k-th closest
// other point (brute force over LDS tiles; the k smallest squared distances of
// each thread are kept sorted in registers).
constexpr int kKnnMax = 32;
__global__ __launch_bounds__(256) void knn_density_kernel(int n, const float* __restrict__ qx,
                                                          const float* __restrict__ qy, int k, float* rho) {
  __shared__ float tx[256], ty[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const float xi = i < n ? qx[i] : 0.f, yi = i < n ? qy[i] : 0.f;
  float best[kKnnMax];
#pragma unroll
  for (int q = 0; q < kKnnMax; ++q) best[q] = INFINITY;
  float kth = INFINITY;  // best[k - 1], kept in a scalar (k is a runtime value)
  for (int j0 = 0; j0 < n; j0 += 256) {
    __syncthreads();
    const int j = j0 + threadIdx.x;
    tx[threadIdx.x] = j < n ? qx[j] : 0.f;
    ty[threadIdx.x] = j < n ? qy[j] : 0.f;
    __syncthreads();
    const int cnt = min(256, n - j0);
    for (int jj = 0; jj < cnt; ++jj) {
      if (j0 + jj == i) continue;
      const float dx = xi - tx[jj], dy = yi - ty[jj];
      float d2 = fmaf(dx, dx, dy * dy);
      if (d2 >= kth) continue;
      // insertion into the sorted list (unrolled; entries beyond k stay unused)
#pragma unroll
      for (int q = 0; q < kKnnMax; ++q) {
        if (q < k && d2 < best[q]) {
          const float t = best[q];
          best[q] = d2;
          d2 = t;
        }
        if (q == k - 1) kth = best[q];
      }
    }
  }
  if (i < n) rho[i] = (float)k / ((float)M_PI * kth);
}

int gauss_product_launch(const GSide& T, const GSide& S, double base_var, double norm, int nrhs, const float* V,
                         int ldv, float* Y, int ldy, float beta, hipStream_t stream) {
  const dim3 grid(cdiv(T.n, kGTile));
  for (int c0 = 0; c0 < nrhs; c0 += kGCols) {
    const int nc = std::min(kGCols, nrhs - c0);
    hipLaunchKernelGGL(gauss_product_kernel, grid, dim3(kGTile), 0, stream, T, S, (float)base_var, (float)norm, nc,
                       V + (size_t)c0 * ldv, ldv, Y + (size_t)c0 * ldy, ldy, beta);
    GPL_LAUNCH_CHECK();
  }
  return GPL_OK;
}

int pixel_shapes_launch(int M, const float* px, const float* py, float* z, hipStream_t stream) {
  hipLaunchKernelGGL(pixel_shapes_kernel, dim3(cdiv(M * M, 256)), dim3(256), 0, stream, M, px, py, z);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" int gpl_gauss_product(const gpl_gauss* g, int nt, const float* tx, const float* ty, const float* tz,
                                 const float* tw, int ns, const float* sx, const float* sy, const float* sz,
                                 const float* sw, int nrhs, const float* V, int ldv, float* Y, int ldy, float beta,
                                 hipStream_t stream) {
  GPL_REQUIRE(g != nullptr, "gauss parameters are NULL");
  GPL_REQUIRE(g->base_var > 0 && std::isfinite(g->base_var) && std::isfinite(g->norm), "base_var must be > 0");
  GPL_REQUIRE(nt >= 0 && ns >= 0 && nrhs >= 0, "negative size");
  if (nt == 0 || nrhs == 0) return GPL_OK;
  GPL_REQUIRE(tx && ty && Y, "NULL target argument");
  GPL_REQUIRE(ns == 0 || (sx && sy && V), "NULL source argument");
  GPL_REQUIRE(ldv >= ns && ldy >= nt, "ldv=%d (>= %d) / ldy=%d (>= %d)", ldv, ns, ldy, nt);
  GPL_REQUIRE(V != Y, "V and Y must not overlap");
  const GSide T{tx, ty, tz, tw, nt}, S{sx, sy, sz, sw, ns};
  return gauss_product_launch(T, S, g->base_var, g->norm, nrhs, V, ldv, Y, ldy, beta, stream);
}

extern "C" int gpl_pixel_shapes(const gpl_grid* grid, const float* px, const float* py, float* z,
                                hipStream_t stream) {
  GPL_REQUIRE(grid != nullptr && grid->n >= 1 && grid->ss >= 1, "bad grid");
  GPL_REQUIRE(px && py && z, "NULL argument");
  return pixel_shapes_launch(grid->n * grid->ss, px, py, z, stream);
}

extern "C" int gpl_knn_density(int n, const float* qx, const float* qy, int k, float* rho, hipStream_t stream) {
  GPL_REQUIRE(k >= 1 && k <= kKnnMax, "k=%d outside [1, %d]", k, kKnnMax);
  GPL_REQUIRE(n > k, "need more than k=%d points, got %d", k, n);
  GPL_REQUIRE(qx && qy && rho, "NULL argument");
  hipLaunchKernelGGL(knn_density_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, qx, qy, k, rho);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
