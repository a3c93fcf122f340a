// Gaussian products with per-point covariances: the pixel-shape (windowed)
// kernel of Sec. 3.2 (eq. "covariance"), the transmission matrix of Sec. 3.4
// (eq. "transmission") and its transpose, and the source reconstruction of
// Sec. 3.5 (eq. "gp-reconstruction"). All are sums
//   Y[i][c] = beta Y[i][c] + norm * wt_i * sum_j ws_j |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2) V[j][c],
//   d = t_i - s_j,  C_ij = Zt_i + Zs_j + base_var I  (2 x 2),
// over target points t and source points s, each optionally with a shape
// covariance Z (three floats: xx, xy, yy) and a weight w. A workgroup owns 64
// targets (one per lane) and runs 8 waves, each over its own eighth of the
// sources, staged 64 at a time in that wave's share of LDS with their
// right-hand-side rows; the 8 partial sums are added in wave order at the end
// (deterministic, and 8 waves per 64 targets fill the chip at tens of thousands
// of points). The Gaussian entries are evaluated in FP32 on the fly and never
// stored. Dense over all pairs (every pair is evaluated).
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace gpl {

constexpr int kGRows = 64;   // targets per workgroup (one per lane)
constexpr int kGWaves = 8;   // waves per workgroup, each over its own share of the sources
constexpr int kGThreads = kGRows * kGWaves;
constexpr int kGCols = 8;    // right-hand-side columns per pass

// |C|^{-1/2} exp(-d^T C^{-1} d / 2) for the 2 x 2 covariance (cxx, cxy; cxy, cyy).
__device__ inline float gauss_pair(float dx, float dy, float cxx, float cxy, float cyy) {
  const float det = fmaf(cxx, cyy, -cxy * cxy);
  const float q = fmaf(cyy * dx, dx, fmaf(-2.f * cxy * dx, dy, cxx * dy * dy)) / det;
  return rsqrtf(det) * exp2_fast(-0.5f * 1.4426950408889634f * q);
}

// 64-point steps of each wave's share of n points: every wave runs the same
// number of steps (so the workgroup barriers are uniform); steps past the end
// are empty.
__device__ inline int wave_steps(int n) { return cdiv(cdiv(n, 64), kGWaves); }

// Shapes on at most one side (kMode 1: targets, or none; kMode 2: sources)
// make C_ij a per-point constant whose inverse and determinant are formed once
// per point; kMode 0 (shapes on both sides, the windowed kernel) forms them per
// pair. NC: right-hand-side columns held per pass (1 or kGCols).
template <int kMode, int NC>
__global__ __launch_bounds__(kGThreads) void gauss_product_kernel(GSide T, GSide S, float base, float norm, int nc,
                                                                  const float* __restrict__ V, int ldv, float* Y,
                                                                  int ldy, float beta) {
  // per source: x, y, then (kMode 0) zxx, zxy, zyy and w, or (kMode 2) the
  // inverse ixx, ixy, iyy and w |C|^{-1/2}, or (kMode 1) w
  __shared__ float sx[kGWaves][64], sy[kGWaves][64], sa[kGWaves][64], sb[kGWaves][64], sc[kGWaves][64],
      sw[kGWaves][64];
  __shared__ float sv[kGWaves][NC][64];
  __shared__ float red[kGWaves - 1][NC][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * kGRows + lane;
  const bool live = i < T.n;
  const float xi = live ? T.x[i] : 0.f, yi = live ? T.y[i] : 0.f;
  const float txx = (live && T.z) ? T.z[i] : 0.f, txy = (live && T.z) ? T.z[T.n + i] : 0.f,
              tyy = (live && T.z) ? T.z[2 * T.n + i] : 0.f;
  float ixx = 0.f, ixy = 0.f, iyy = 0.f, rdet = 1.f;
  if (kMode == 1) {
    const float cxx = txx + base, cxy = txy, cyy = tyy + base;
    const float det = fmaf(cxx, cyy, -cxy * cxy), idet = 1.f / det;
    ixx = cyy * idet;
    ixy = -cxy * idet;
    iyy = cxx * idet;
    rdet = rsqrtf(det);
  }
  const float kq = -0.5f * 1.4426950408889634f;
  float acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.f;
  const int steps = wave_steps(S.n);
  for (int st = 0; st < steps; ++st) {
    const int j0 = (wv * steps + st) * 64;
    __syncthreads();
    const int j = j0 + lane;
    const bool sj = j < S.n;
    const float zxx = (sj && S.z) ? S.z[j] : 0.f, zxy = (sj && S.z) ? S.z[S.n + j] : 0.f,
                zyy = (sj && S.z) ? S.z[2 * S.n + j] : 0.f;
    const float wj = sj ? (S.w ? S.w[j] : 1.f) : 0.f;
    sx[wv][lane] = sj ? S.x[j] : 0.f;
    sy[wv][lane] = sj ? S.y[j] : 0.f;
    if (kMode == 2) {
      const float cxx = zxx + base, cxy = zxy, cyy = zyy + base;
      const float det = fmaf(cxx, cyy, -cxy * cxy), idet = 1.f / det;
      sa[wv][lane] = cyy * idet;
      sb[wv][lane] = -cxy * idet;
      sc[wv][lane] = cxx * idet;
      sw[wv][lane] = wj * rsqrtf(det);
    } else {
      sa[wv][lane] = zxx;
      sb[wv][lane] = zxy;
      sc[wv][lane] = zyy;
      sw[wv][lane] = wj;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) sv[wv][c][lane] = (sj && c < nc) ? V[(size_t)c * ldv + j] : 0.f;
    __syncthreads();
    const int cnt = max(0, min(64, S.n - j0));
    for (int jj = 0; jj < cnt; ++jj) {
      const float dx = xi - sx[wv][jj], dy = yi - sy[wv][jj];
      float val;
      if (kMode == 0) {
        val = sw[wv][jj] * gauss_pair(dx, dy, txx + sa[wv][jj] + base, txy + sb[wv][jj], tyy + sc[wv][jj] + base);
      } else {
        const float a = kMode == 2 ? sa[wv][jj] : ixx, b = kMode == 2 ? sb[wv][jj] : ixy,
                    c = kMode == 2 ? sc[wv][jj] : iyy;
        const float ux = fmaf(a, dx, b * dy), uy = fmaf(b, dx, c * dy);
        val = sw[wv][jj] * exp2_fast(kq * fmaf(dx, ux, dy * uy));
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = fmaf(val, sv[wv][c][jj], acc[c]);
    }
  }
  if (wv > 0)
#pragma unroll
    for (int c = 0; c < NC; ++c) red[wv - 1][c][lane] = acc[c];
  __syncthreads();
  if (wv > 0 || !live) return;
  for (int w = 0; w < kGWaves - 1; ++w)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += red[w][c][lane];
  const float f = norm * (T.w ? T.w[i] : 1.f) * rdet;
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

// Adjoint of one column of the Gaussian product. With
//   F = sum_i U_i norm wt_i sum_j ws_j V_j G_ij,  G_ij = |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2),
// d = t_i - s_j, dG/dd = -G C^{-1} d and dG/dC = G (C^{-1} d d^T C^{-1} - C^{-1}) / 2:
// the target pass accumulates gtx/gty += dF/dt_i and (optionally) gtz += dF/dZt_i
// as the symmetric matrix gradient (xx, xy, yy entries); the source pass
// accumulates gsx/gsy += dF/ds_j and gsw += dF/dws_j. Sources without shapes
// only (their shape gradient is not formed).
template <bool kShapes>
__global__ __launch_bounds__(kGThreads) void gauss_backward_target_kernel(GSide T, GSide S, float base, float norm,
                                                                          const float* __restrict__ V,
                                                                          const float* __restrict__ U, float* gtx,
                                                                          float* gty, float* gtz) {
  constexpr int kAcc = kShapes ? 6 : 2;
  __shared__ float sx[kGWaves][64], sy[kGWaves][64], swv[kGWaves][64];
  __shared__ float red[kGWaves - 1][kAcc][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * kGRows + lane;
  const bool live = i < T.n;
  const float xi = live ? T.x[i] : 0.f, yi = live ? T.y[i] : 0.f;
  const float txx = (live && T.z) ? T.z[i] : 0.f, txy = (live && T.z) ? T.z[T.n + i] : 0.f,
              tyy = (live && T.z) ? T.z[2 * T.n + i] : 0.f;
  // the source side has no shapes: C = Zt_i + base I is fixed per target
  const float cxx = txx + base, cxy = txy, cyy = tyy + base;
  const float det = fmaf(cxx, cyy, -cxy * cxy), idet = 1.f / det, rdet = rsqrtf(det);
  const float ixx = cyy * idet, ixy = -cxy * idet, iyy = cxx * idet;
  float acc[kAcc];  // ax, ay, then (shapes) sum g, zxx, zxy, zyy
#pragma unroll
  for (int a = 0; a < kAcc; ++a) acc[a] = 0.f;
  const int steps = wave_steps(S.n);
  for (int st = 0; st < steps; ++st) {
    const int j0 = (wv * steps + st) * 64;
    __syncthreads();
    const int j = j0 + lane;
    const bool sj = j < S.n;
    sx[wv][lane] = sj ? S.x[j] : 0.f;
    sy[wv][lane] = sj ? S.y[j] : 0.f;
    swv[wv][lane] = sj ? (S.w ? S.w[j] : 1.f) * V[j] : 0.f;
    __syncthreads();
    const int cnt = max(0, min(64, S.n - j0));
    for (int jj = 0; jj < cnt; ++jj) {
      const float dx = xi - sx[wv][jj], dy = yi - sy[wv][jj];
      const float ux = fmaf(ixx, dx, ixy * dy), uy = fmaf(ixy, dx, iyy * dy);
      const float q = fmaf(dx, ux, dy * uy);
      const float gv = swv[wv][jj] * exp2_fast(-0.5f * 1.4426950408889634f * q);
      acc[0] = fmaf(gv, ux, acc[0]);
      acc[1] = fmaf(gv, uy, acc[1]);
      if (kShapes) {
        acc[2 % kAcc] += gv;
        acc[3 % kAcc] = fmaf(gv * ux, ux, acc[3 % kAcc]);
        acc[4 % kAcc] = fmaf(gv * ux, uy, acc[4 % kAcc]);
        acc[5 % kAcc] = fmaf(gv * uy, uy, acc[5 % kAcc]);
      }
    }
  }
  if (wv > 0)
#pragma unroll
    for (int a = 0; a < kAcc; ++a) red[wv - 1][a][lane] = acc[a];
  __syncthreads();
  if (wv > 0 || !live) return;
  for (int w = 0; w < kGWaves - 1; ++w)
#pragma unroll
    for (int a = 0; a < kAcc; ++a) acc[a] += red[w][a][lane];
  const float c = norm * (T.w ? T.w[i] : 1.f) * U[i] * rdet;
  gtx[i] -= c * acc[0];
  gty[i] -= c * acc[1];
  if (kShapes) {
    const float h = 0.5f * c;
    gtz[i] += h * (acc[3 % kAcc] - ixx * acc[2 % kAcc]);
    gtz[T.n + i] += h * (acc[4 % kAcc] - ixy * acc[2 % kAcc]);
    gtz[2 * T.n + i] += h * (acc[5 % kAcc] - iyy * acc[2 % kAcc]);
  }
}

__global__ __launch_bounds__(kGThreads) void gauss_backward_source_kernel(GSide T, GSide S, float base, float norm,
                                                                          const float* __restrict__ V,
                                                                          const float* __restrict__ U, float* gsx,
                                                                          float* gsy, float* gsw) {
  // per target: position, the inverse of C_i = Zt_i + base I, and wt_i U_i |C_i|^{-1/2}
  __shared__ float tx[kGWaves][64], ty[kGWaves][64], ta[kGWaves][64], tb[kGWaves][64], tcc[kGWaves][64],
      tc[kGWaves][64];
  __shared__ float red[kGWaves - 1][3][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.x * kGRows + lane;
  const bool live = j < S.n;
  const float xj = live ? S.x[j] : 0.f, yj = live ? S.y[j] : 0.f;
  const float kq = -0.5f * 1.4426950408889634f;
  float ax = 0.f, ay = 0.f, aw = 0.f;
  const int steps = wave_steps(T.n);
  for (int st = 0; st < steps; ++st) {
    const int i0 = (wv * steps + st) * 64;
    __syncthreads();
    const int i = i0 + lane;
    const bool ti = i < T.n;
    const float cxx = ((ti && T.z) ? T.z[i] : 0.f) + base, cxy = (ti && T.z) ? T.z[T.n + i] : 0.f,
                cyy = ((ti && T.z) ? T.z[2 * T.n + i] : 0.f) + base;
    const float det = fmaf(cxx, cyy, -cxy * cxy), idet = 1.f / det;
    tx[wv][lane] = ti ? T.x[i] : 0.f;
    ty[wv][lane] = ti ? T.y[i] : 0.f;
    ta[wv][lane] = cyy * idet;
    tb[wv][lane] = -cxy * idet;
    tcc[wv][lane] = cxx * idet;
    tc[wv][lane] = ti ? (T.w ? T.w[i] : 1.f) * U[i] * rsqrtf(det) : 0.f;
    __syncthreads();
    const int cnt = max(0, min(64, T.n - i0));
    for (int ii = 0; ii < cnt; ++ii) {
      const float dx = tx[wv][ii] - xj, dy = ty[wv][ii] - yj;
      const float ixx = ta[wv][ii], ixy = tb[wv][ii], iyy = tcc[wv][ii];
      const float ux = fmaf(ixx, dx, ixy * dy), uy = fmaf(ixy, dx, iyy * dy);
      const float gv = tc[wv][ii] * exp2_fast(kq * fmaf(dx, ux, dy * uy));
      ax = fmaf(gv, ux, ax);
      ay = fmaf(gv, uy, ay);
      aw += gv;
    }
  }
  if (wv > 0) {
    red[wv - 1][0][lane] = ax;
    red[wv - 1][1][lane] = ay;
    red[wv - 1][2][lane] = aw;
  }
  __syncthreads();
  if (wv > 0 || !live) return;
  for (int w = 0; w < kGWaves - 1; ++w) {
    ax += red[w][0][lane];
    ay += red[w][1][lane];
    aw += red[w][2][lane];
  }
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
      hipLaunchKernelGGL(gauss_backward_target_kernel<true>, dim3(cdiv(T.n, kGRows)), dim3(kGThreads), 0, stream, T, S,
                         (float)base_var, (float)norm, V, U, gtx, gty, gtz);
    else
      hipLaunchKernelGGL(gauss_backward_target_kernel<false>, dim3(cdiv(T.n, kGRows)), dim3(kGThreads), 0, stream, T,
                         S, (float)base_var, (float)norm, V, U, gtx, gty, gtz);
    GPL_LAUNCH_CHECK();
  }
  if (gsx || gsw) {
    hipLaunchKernelGGL(gauss_backward_source_kernel, dim3(cdiv(S.n, kGRows)), dim3(kGThreads), 0, stream, T, S,
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
  const dim3 grid(cdiv(T.n, kGRows));
  const int mode = S.z == nullptr ? 1 : (T.z == nullptr ? 2 : 0);
  for (int c0 = 0; c0 < nrhs; c0 += kGCols) {
    const int nc = std::min(kGCols, nrhs - c0);
    const float *v = V + (size_t)c0 * ldv;
    float* y = Y + (size_t)c0 * ldy;
    const float b = (float)base_var, nm = (float)norm;
#define GPL_GAUSS_LAUNCH(M, C) \
  hipLaunchKernelGGL((gauss_product_kernel<M, C>), grid, dim3(kGThreads), 0, stream, T, S, b, nm, nc, v, ldv, y, ldy, beta)
    if (nc == 1) {
      if (mode == 0) GPL_GAUSS_LAUNCH(0, 1);
      else if (mode == 1) GPL_GAUSS_LAUNCH(1, 1);
      else GPL_GAUSS_LAUNCH(2, 1);
    } else {
      if (mode == 0) GPL_GAUSS_LAUNCH(0, kGCols);
      else if (mode == 1) GPL_GAUSS_LAUNCH(1, kGCols);
      else GPL_GAUSS_LAUNCH(2, kGCols);
    }
#undef GPL_GAUSS_LAUNCH
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
