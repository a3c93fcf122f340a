// Distance to the k-th closest other point, for the density of inducing points
// of the transmission weights (Sec. 3.4, footnote to eq. "transmission": the
// area of the circle reaching the k-th closest point, k = 20).
//
// The points are sorted along the Hilbert curve of the tile plan and grouped in
// 32-point chunks with bounding boxes. A wave (64 consecutive sorted points)
// first takes the chunks near its own in curve order, which bounds each lane's
// k-th distance, then visits only the chunks whose box some lane can still
// reach within its bound. Candidates are ranked by squared distance in FP32,
// equal distances by the lower caller index.
#include <climits>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"
#include "tileplan.hpp"

namespace gpl {

constexpr int kKnnMaxK = 32;
constexpr int kKnnNear = 6;  // chunks on each side of a wave's own two taken first

__device__ inline bool knn_before(float d, int id, float bd, int bid) { return d < bd || (d == bd && id < bid); }

__global__ __launch_bounds__(256) void knn_sorted_kernel(int n, int nch, const float* __restrict__ xs,
                                                         const float* __restrict__ ys, const int* __restrict__ perm,
                                                         const float4* __restrict__ cbox, int k, float* rho,
                                                         float* rk, int* nn) {
  const int i = blockIdx.x * 256 + threadIdx.x;  // sorted position
  const bool live = i < n;
  const float xi = live ? xs[i] : 0.f, yi = live ? ys[i] : 0.f;
  const int me = live ? perm[i] : -1;
  float best[kKnnMaxK];
  int bid[kKnnMaxK];
#pragma unroll
  for (int q = 0; q < kKnnMaxK; ++q) {
    best[q] = INFINITY;
    bid[q] = INT_MAX;
  }
  float kth = INFINITY;  // best[k - 1] and its index, kept in scalars (k is a runtime value)
  int kid = INT_MAX;
  auto visit = [&](int c) {
    const int j0 = c * kChunk;
    const int cnt = min(kChunk, n - j0);
    for (int jj = 0; jj < cnt; ++jj) {
      const int j = j0 + jj;
      const float dx = xi - xs[j], dy = yi - ys[j];
      float d2 = fmaf(dx, dx, dy * dy);
      int id = perm[j];
      if (!live || id == me || !knn_before(d2, id, kth, kid)) continue;
#pragma unroll
      for (int q = 0; q < kKnnMaxK; ++q) {
        if (q < k && knn_before(d2, id, best[q], bid[q])) {
          const float t = best[q];
          const int ti = bid[q];
          best[q] = d2;
          bid[q] = id;
          d2 = t;
          id = ti;
        }
        if (q == k - 1) {
          kth = best[q];
          kid = bid[q];
        }
      }
    }
  };
  const int cw = (blockIdx.x * 256 + (threadIdx.x & ~63)) / kChunk;  // the wave's first chunk
  const int lo = max(0, cw - kKnnNear), hi = min(nch, cw + 2 + kKnnNear);
  for (int c = lo; c < hi; ++c) visit(c);
  for (int c = 0; c < nch; ++c) {
    if (c >= lo && c < hi) continue;
    const float4 b = cbox[c];
    const float gx = fmaxf(0.f, fmaxf(b.x - xi, xi - b.y));
    const float gy = fmaxf(0.f, fmaxf(b.z - yi, yi - b.w));
    const bool need = live && fmaf(gx, gx, gy * gy) <= kth;
    if (__ballot(need) == 0ull) continue;  // no lane of the wave can reach this chunk
    visit(c);
  }
  if (!live) return;
  if (rho) rho[me] = (float)k / ((float)M_PI * kth);
  if (rk) rk[me] = sqrtf(kth);
  if (nn) nn[me] = kid;
}

size_t knn_workspace(int n) { return plan_workspace(n); }

int knn_index_launch(int n, const float* qx, const float* qy, int k, float* rho, float* rk, int* nn, void* ws,
                     size_t ws_bytes, hipStream_t stream) {
  GPL_REQUIRE(k >= 1 && k <= kKnnMaxK && n > k, "k=%d must be in [1, %d] and below n=%d", k, kKnnMaxK, n);
  GPL_TRY(check_ws(ws, ws_bytes, knn_workspace(n)));
  Carver cv(ws, ws_bytes);
  TilePlan p;
  plan_carve(cv, n, p);
  GPL_REQUIRE(cv.ok(), "workspace too small for the point sort");
  GPL_TRY(plan_sort(p, n, qx, qy, stream));
  hipLaunchKernelGGL(knn_sorted_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, p.nch, p.xs, p.ys, p.perm,
                     p.cbox, k, rho, rk, nn);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" size_t gpl_knn_density_workspace(int n) { return n <= 0 ? 0 : knn_workspace(n); }

extern "C" int gpl_knn_density(int n, const float* qx, const float* qy, int k, float* rho, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  GPL_REQUIRE(qx && qy && rho, "NULL argument");
  return knn_index_launch(n, qx, qy, k, rho, nullptr, nullptr, ws, ws_bytes, stream);
}
