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

// |C|^{-1/2} exp(-d^T C^{-1} d / 2) for the 2 x 2 covariance (cxx, cxy; cxy, cyy).
__device__ inline float gauss_pair(float dx, float dy, float cxx, float cxy, float cyy) {
  const float det = fmaf(cxx, cyy, -cxy * cxy);
  const float q = fmaf(cyy * dx, dx, fmaf(-2.f * cxy * dx, dy, cxx * dy * dy)) / det;
  return rsqrtf(det) * exp2_fast(-0.5f * 1.4426950408889634f * q);
}

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
      const float val = sw[jj] * gauss_pair(xi - sx[jj], yi - sy[jj], txx + sxx[jj] + base, txy + sxy[jj],
                                            tyy + syy[jj] + base);
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

// The same Gaussian entries written out as a dense nt x ns matrix (column-major,
// ld ldm): M[j*ldm + i] = norm wt_i ws_j |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2).
// Block b covers targets 256 (b mod ntb) .. +255 of source b / ntb, so each
// column is written by coalesced stores.
__global__ __launch_bounds__(256) void gauss_matrix_kernel(GSide T, GSide S, float base, float norm, int ntb,
                                                           float* M, int ldm) {
  const int tb = blockIdx.x % ntb, j = blockIdx.x / ntb;
  const int i = tb * 256 + threadIdx.x;
  if (i >= T.n) return;
  const float txx = T.z ? T.z[i] : 0.f, txy = T.z ? T.z[T.n + i] : 0.f, tyy = T.z ? T.z[2 * T.n + i] : 0.f;
  const float sxx = S.z ? S.z[j] : 0.f, sxy = S.z ? S.z[S.n + j] : 0.f, syy = S.z ? S.z[2 * S.n + j] : 0.f;
  const float w = norm * (T.w ? T.w[i] : 1.f) * (S.w ? S.w[j] : 1.f);
  M[(size_t)j * ldm + i] = w * gauss_pair(T.x[i] - S.x[j], T.y[i] - S.y[j], txx + sxx + base, txy + sxy,
                                          tyy + syy + base);
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
// kIndex: also keep the neighbours' indices and write, per point, the distance
// r_k and the index of its k-th closest other point (equal distances keep the
// lower index first).
template <bool kIndex>
__global__ __launch_bounds__(256) void knn_kernel(int n, const float* __restrict__ qx, const float* __restrict__ qy,
                                                  int k, float* rho, float* rk, int* nn) {
  __shared__ float tx[256], ty[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const float xi = i < n ? qx[i] : 0.f, yi = i < n ? qy[i] : 0.f;
  float best[kKnnMax];
  int bidx[kIndex ? kKnnMax : 1];
#pragma unroll
  for (int q = 0; q < kKnnMax; ++q) best[q] = INFINITY;
  if (kIndex)
#pragma unroll
    for (int q = 0; q < kKnnMax; ++q) bidx[kIndex ? q : 0] = -1;
  float kth = INFINITY;  // best[k - 1], kept in a scalar (k is a runtime value)
  int kidx = -1;
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
      int id = j0 + jj;
      // insertion into the sorted list (unrolled; entries beyond k stay unused)
#pragma unroll
      for (int q = 0; q < kKnnMax; ++q) {
        if (q < k && d2 < best[q]) {
          const float t = best[q];
          best[q] = d2;
          d2 = t;
          if (kIndex) {
            const int ti = bidx[kIndex ? q : 0];
            bidx[kIndex ? q : 0] = id;
            id = ti;
          }
        }
        if (q == k - 1) {
          kth = best[q];
          if (kIndex) kidx = bidx[kIndex ? q : 0];
        }
      }
    }
  }
  if (i >= n) return;
  if (rho) rho[i] = (float)k / ((float)M_PI * kth);
  if (kIndex) {
    rk[i] = sqrtf(kth);
    nn[i] = kidx;
  }
}

// Adjoint of one column of the Gaussian product. With
//   F = sum_i U_i norm wt_i sum_j ws_j V_j G_ij,  G_ij = |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2),
// d = t_i - s_j, dG/dd = -G C^{-1} d and dG/dC = G (C^{-1} d d^T C^{-1} - C^{-1}) / 2:
// the target pass accumulates gtx/gty += dF/dt_i and (optionally) gtz += dF/dZt_i
// as the symmetric matrix gradient (xx, xy, yy entries); the source pass
// accumulates gsx/gsy += dF/ds_j and gsw += dF/dws_j. Sources without shapes
// only (their shape gradient is not formed).
template <bool kShapes>
__global__ __launch_bounds__(kGTile) void gauss_backward_target_kernel(GSide T, GSide S, float base, float norm,
                                                                       const float* __restrict__ V,
                                                                       const float* __restrict__ U, float* gtx,
                                                                       float* gty, float* gtz) {
  __shared__ float sx[kGTile], sy[kGTile], swv[kGTile];
  const int i = blockIdx.x * kGTile + threadIdx.x;
  const bool live = i < T.n;
  const float xi = live ? T.x[i] : 0.f, yi = live ? T.y[i] : 0.f;
  const float txx = (live && T.z) ? T.z[i] : 0.f, txy = (live && T.z) ? T.z[T.n + i] : 0.f,
              tyy = (live && T.z) ? T.z[2 * T.n + i] : 0.f;
  // the source side has no shapes: C = Zt_i + base I is fixed per target
  const float cxx = txx + base, cxy = txy, cyy = tyy + base;
  const float det = fmaf(cxx, cyy, -cxy * cxy), idet = 1.f / det, rdet = rsqrtf(det);
  const float ixx = cyy * idet, ixy = -cxy * idet, iyy = cxx * idet;
  float ax = 0.f, ay = 0.f, zs = 0.f, zxx = 0.f, zxy = 0.f, zyy = 0.f;
  for (int j0 = 0; j0 < S.n; j0 += kGTile) {
    __syncthreads();
    const int j = j0 + threadIdx.x;
    const bool sj = j < S.n;
    sx[threadIdx.x] = sj ? S.x[j] : 0.f;
    sy[threadIdx.x] = sj ? S.y[j] : 0.f;
    swv[threadIdx.x] = sj ? (S.w ? S.w[j] : 1.f) * V[j] : 0.f;
    __syncthreads();
    const int cnt = min(kGTile, S.n - j0);
    for (int jj = 0; jj < cnt; ++jj) {
      const float dx = xi - sx[jj], dy = yi - sy[jj];
      const float ux = fmaf(ixx, dx, ixy * dy), uy = fmaf(ixy, dx, iyy * dy);
      const float q = fmaf(dx, ux, dy * uy);
      const float gv = swv[jj] * exp2_fast(-0.5f * 1.4426950408889634f * q);
      ax = fmaf(gv, ux, ax);
      ay = fmaf(gv, uy, ay);
      if (kShapes) {
        zs += gv;
        zxx = fmaf(gv * ux, ux, zxx);
        zxy = fmaf(gv * ux, uy, zxy);
        zyy = fmaf(gv * uy, uy, zyy);
      }
    }
  }
  if (!live) return;
  const float c = norm * (T.w ? T.w[i] : 1.f) * U[i] * rdet;
  gtx[i] -= c * ax;
  gty[i] -= c * ay;
  if (kShapes) {
    const float h = 0.5f * c;
    gtz[i] += h * (zxx - ixx * zs);
    gtz[T.n + i] += h * (zxy - ixy * zs);
    gtz[2 * T.n + i] += h * (zyy - iyy * zs);
  }
}

__global__ __launch_bounds__(kGTile) void gauss_backward_source_kernel(GSide T, GSide S, float base, float norm,
                                                                       const float* __restrict__ V,
                                                                       const float* __restrict__ U, float* gsx,
                                                                       float* gsy, float* gsw) {
  __shared__ float tx[kGTile], ty[kGTile], txx[kGTile], txy[kGTile], tyy[kGTile], tc[kGTile];
  const int j = blockIdx.x * kGTile + threadIdx.x;
  const bool live = j < S.n;
  const float xj = live ? S.x[j] : 0.f, yj = live ? S.y[j] : 0.f;
  float ax = 0.f, ay = 0.f, aw = 0.f;
  for (int i0 = 0; i0 < T.n; i0 += kGTile) {
    __syncthreads();
    const int i = i0 + threadIdx.x;
    const bool ti = i < T.n;
    tx[threadIdx.x] = ti ? T.x[i] : 0.f;
    ty[threadIdx.x] = ti ? T.y[i] : 0.f;
    txx[threadIdx.x] = (ti && T.z) ? T.z[i] : 0.f;
    txy[threadIdx.x] = (ti && T.z) ? T.z[T.n + i] : 0.f;
    tyy[threadIdx.x] = (ti && T.z) ? T.z[2 * T.n + i] : 0.f;
    tc[threadIdx.x] = ti ? (T.w ? T.w[i] : 1.f) * U[i] : 0.f;
    __syncthreads();
    const int cnt = min(kGTile, T.n - i0);
    for (int ii = 0; ii < cnt; ++ii) {
      const float cxx = txx[ii] + base, cxy = txy[ii], cyy = tyy[ii] + base;
      const float idet = 1.f / fmaf(cxx, cyy, -cxy * cxy);
      const float ixx = cyy * idet, ixy = -cxy * idet, iyy = cxx * idet;
      const float dx = tx[ii] - xj, dy = ty[ii] - yj;
      const float ux = fmaf(ixx, dx, ixy * dy), uy = fmaf(ixy, dx, iyy * dy);
      const float q = fmaf(dx, ux, dy * uy);
      const float gv = tc[ii] * sqrtf(idet) * exp2_fast(-0.5f * 1.4426950408889634f * q);
      ax = fmaf(gv, ux, ax);
      ay = fmaf(gv, uy, ay);
      aw += gv;
    }
  }
  if (!live) return;
  const float f = norm * V[j];
  const float fw = f * (S.w ? S.w[j] : 1.f);
  if (gsx) {
    gsx[j] += fw * ax;
    gsy[j] += fw * ay;
  }
  if (gsw) gsw[j] += f * aw;
}

// Adjoint of pixel_shapes: gz holds dF/dZ_j as a symmetric matrix gradient;
// Z = (a a^T + b b^T) / (4 pi) gives dF/da = Gbar a / (2 pi), likewise for b.
// First pass: per point, (dF/da, dF/db) into gab (4 arrays of M*M floats).
__global__ void pixel_axes_grad_kernel(int M, const float* __restrict__ px, const float* __restrict__ py,
                                       const float* __restrict__ gz, float* gab) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = M * M;
  if (j >= N) return;
  const int fy = j / M, fx = j - fy * M;
  float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
  if (M > 1) {
    auto diff = [&](int lo, int hi, float h) { return make_float2((px[hi] - px[lo]) * h, (py[hi] - py[lo]) * h); };
    if (fx == 0) a = diff(j, j + 1, 1.f);
    else if (fx == M - 1) a = diff(j - 1, j, 1.f);
    else a = diff(j - 1, j + 1, 0.5f);
    if (fy == 0) b = diff(j, j + M, 1.f);
    else if (fy == M - 1) b = diff(j - M, j, 1.f);
    else b = diff(j - M, j + M, 0.5f);
  }
  const float f = (float)(1.0 / (2.0 * M_PI));
  const float gxx = gz[j], gxy = gz[N + j], gyy = gz[2 * N + j];
  gab[j] = f * fmaf(gxx, a.x, gxy * a.y);
  gab[N + j] = f * fmaf(gxy, a.x, gyy * a.y);
  gab[2 * N + j] = f * fmaf(gxx, b.x, gxy * b.y);
  gab[3 * N + j] = f * fmaf(gxy, b.x, gyy * b.y);
}

// d a_c / d p_m along one grid line of length M (one-sided differences at the ends).
__device__ inline float axis_coef(int c, int m, int M) {
  if (M == 1) return 0.f;
  if (c == 0) return (m == 1 ? 1.f : 0.f) - (m == 0 ? 1.f : 0.f);
  if (c == M - 1) return (m == M - 1 ? 1.f : 0.f) - (m == M - 2 ? 1.f : 0.f);
  return (m == c + 1 ? 0.5f : 0.f) - (m == c - 1 ? 0.5f : 0.f);
}

// Second pass: gpx/gpy[m] += sum over the axes that depend on p_m (neighbours
// c = m-1, m, m+1 along the row for a, along the column for b).
__global__ void pixel_axes_gather_kernel(int M, const float* __restrict__ gab, float* gpx, float* gpy) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = M * M;
  if (m >= N) return;
  const int fy = m / M, fx = m - fy * M;
  float sx = 0.f, sy = 0.f;
  for (int c = max(fx - 1, 0); c <= min(fx + 1, M - 1); ++c) {
    const float w = axis_coef(c, fx, M);
    const int j = fy * M + c;
    sx = fmaf(w, gab[j], sx);
    sy = fmaf(w, gab[N + j], sy);
  }
  for (int c = max(fy - 1, 0); c <= min(fy + 1, M - 1); ++c) {
    const float w = axis_coef(c, fy, M);
    const int j = c * M + fx;
    sx = fmaf(w, gab[2 * N + j], sx);
    sy = fmaf(w, gab[3 * N + j], sy);
  }
  gpx[m] += sx;
  gpy[m] += sy;
}

// Adjoint of weights w_j = r_j sqrt(pi / k) (w = rho^{-1/2}, rho = k / (pi r^2)),
// r_j = |q_j - q_nn(j)|: dF/dq_j += coef v, dF/dq_nn(j) -= coef v with
// v = q_j - q_nn(j), coef = gw_j w_j / r_j^2. The neighbour's share is
// scattered with FP64 atomic adds into gq (2n doubles: x then y).
__global__ void knn_weight_backward_kernel(int n, const float* __restrict__ qx, const float* __restrict__ qy,
                                           const float* __restrict__ rk, const int* __restrict__ nn,
                                           const float* __restrict__ w, const float* __restrict__ gw, double* gq) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int o = nn[j];
  const float r = rk[j];
  if (o < 0 || !(r > 0.f)) return;
  const double coef = (double)gw[j] * (double)w[j] / ((double)r * (double)r);
  const double vx = coef * (double)(qx[j] - qx[o]), vy = coef * (double)(qy[j] - qy[o]);
  atomicAdd(gq + j, vx);
  atomicAdd(gq + n + j, vy);
  atomicAdd(gq + o, -vx);
  atomicAdd(gq + n + o, -vy);
}

__global__ void add_double_pairs_kernel(int n, const double* __restrict__ gq, float* gpx, float* gpy) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  gpx[j] += (float)gq[j];
  gpy[j] += (float)gq[n + j];
}

int gauss_backward_launch(const GSide& T, const GSide& S, double base_var, double norm, const float* V, const float* U,
                          float* gtx, float* gty, float* gtz, float* gsx, float* gsy, float* gsw, hipStream_t stream) {
  GPL_REQUIRE(S.z == nullptr, "the adjoint supports sources without shape covariances");
  if (T.n == 0 || S.n == 0) return GPL_OK;
  if (gtx) {
    if (gtz)
      hipLaunchKernelGGL(gauss_backward_target_kernel<true>, dim3(cdiv(T.n, kGTile)), dim3(kGTile), 0, stream, T, S,
                         (float)base_var, (float)norm, V, U, gtx, gty, gtz);
    else
      hipLaunchKernelGGL(gauss_backward_target_kernel<false>, dim3(cdiv(T.n, kGTile)), dim3(kGTile), 0, stream, T,
                         S, (float)base_var, (float)norm, V, U, gtx, gty, gtz);
    GPL_LAUNCH_CHECK();
  }
  if (gsx || gsw) {
    hipLaunchKernelGGL(gauss_backward_source_kernel, dim3(cdiv(S.n, kGTile)), dim3(kGTile), 0, stream, T, S,
                       (float)base_var, (float)norm, V, U, gsx, gsy, gsw);
    GPL_LAUNCH_CHECK();
  }
  return GPL_OK;
}

int pixel_shapes_backward_launch(int M, const float* px, const float* py, const float* gz, float* gab, float* gpx,
                                 float* gpy, hipStream_t stream) {
  const int N = M * M;
  hipLaunchKernelGGL(pixel_axes_grad_kernel, dim3(cdiv(N, 256)), dim3(256), 0, stream, M, px, py, gz, gab);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(pixel_axes_gather_kernel, dim3(cdiv(N, 256)), dim3(256), 0, stream, M, gab, gpx, gpy);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int knn_index_launch(int n, const float* qx, const float* qy, int k, float* rho, float* rk, int* nn,
                     hipStream_t stream) {
  GPL_REQUIRE(k >= 1 && k <= kKnnMax && n > k, "k=%d must be in [1, %d] and below n=%d", k, kKnnMax, n);
  hipLaunchKernelGGL(knn_kernel<true>, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, qx, qy, k, rho, rk, nn);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int knn_weight_backward_launch(int n, const float* qx, const float* qy, const float* rk, const int* nn,
                               const float* w, const float* gw, double* gq, float* gpx, float* gpy,
                               hipStream_t stream) {
  hipLaunchKernelGGL(knn_weight_backward_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, qx, qy, rk, nn, w, gw,
                     gq);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(add_double_pairs_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, gq, gpx, gpy);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
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

extern "C" int gpl_gauss_matrix(const gpl_gauss* g, int nt, const float* tx, const float* ty, const float* tz,
                                const float* tw, int ns, const float* sx, const float* sy, const float* sz,
                                const float* sw, float* M, int ldm, hipStream_t stream) {
  GPL_REQUIRE(g != nullptr, "gauss parameters are NULL");
  GPL_REQUIRE(g->base_var > 0 && std::isfinite(g->base_var) && std::isfinite(g->norm), "base_var must be > 0");
  GPL_REQUIRE(nt >= 0 && ns >= 0, "negative size");
  if (nt == 0 || ns == 0) return GPL_OK;
  GPL_REQUIRE(tx && ty && sx && sy && M, "NULL argument");
  GPL_REQUIRE(ldm >= nt, "ldm=%d must be >= nt=%d", ldm, nt);
  const int ntb = cdiv(nt, 256);
  GPL_REQUIRE((long long)ntb * ns <= 0x7fffffffLL, "matrix too large for one launch");
  const GSide T{tx, ty, tz, tw, nt}, S{sx, sy, sz, sw, ns};
  hipLaunchKernelGGL(gauss_matrix_kernel, dim3(ntb * ns), dim3(256), 0, stream, T, S, (float)g->base_var,
                     (float)g->norm, ntb, M, ldm);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" int gpl_gauss_product_backward(const gpl_gauss* g, int nt, const float* tx, const float* ty,
                                         const float* tz, const float* tw, int ns, const float* sx, const float* sy,
                                         const float* sw, const float* V, const float* U, float* gtx, float* gty,
                                         float* gtz, float* gsx, float* gsy, float* gsw, hipStream_t stream) {
  GPL_REQUIRE(g != nullptr, "gauss parameters are NULL");
  GPL_REQUIRE(g->base_var > 0 && std::isfinite(g->base_var) && std::isfinite(g->norm), "base_var must be > 0");
  GPL_REQUIRE(nt >= 0 && ns >= 0, "negative size");
  if (nt == 0 || ns == 0) return GPL_OK;
  GPL_REQUIRE(tx && ty && sx && sy && V && U, "NULL input");
  GPL_REQUIRE((gtx == nullptr) == (gty == nullptr) && (gsx == nullptr) == (gsy == nullptr), "gradient pairs");
  GPL_REQUIRE(gtz == nullptr || (gtx != nullptr && tz != nullptr), "gtz needs gtx and target shapes");
  const GSide T{tx, ty, tz, tw, nt}, S{sx, sy, nullptr, sw, ns};
  return gauss_backward_launch(T, S, g->base_var, g->norm, V, U, gtx, gty, gtz, gsx, gsy, gsw, stream);
}

extern "C" int gpl_pixel_shapes_backward(const gpl_grid* grid, const float* px, const float* py, const float* gz,
                                         float* gpx, float* gpy, void* ws, size_t ws_bytes, hipStream_t stream) {
  GPL_REQUIRE(grid != nullptr && grid->n >= 1 && grid->ss >= 1, "bad grid");
  GPL_REQUIRE(px && py && gz && gpx && gpy, "NULL argument");
  const int M = grid->n * grid->ss;
  GPL_TRY(check_ws(ws, ws_bytes, align_up(sizeof(float) * 4 * (size_t)M * M)));
  return pixel_shapes_backward_launch(M, px, py, gz, static_cast<float*>(ws), gpx, gpy, stream);
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
  hipLaunchKernelGGL(knn_kernel<false>, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, qx, qy, k, rho, nullptr,
                     nullptr);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
