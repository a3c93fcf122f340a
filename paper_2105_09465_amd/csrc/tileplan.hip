// Construction of the tile plan of the kernel product (see tileplan.hpp): sorted
// points, chunk bounding boxes, and per row tile the list of chunks within the
// exact-zero cutoff of the kernel (Sec. 3.1, eq. "grbf").
#include <cmath>

#include "tileplan.hpp"

namespace gpl {

size_t plan_workspace(int n) {
  if (n <= 0) return 0;
  Sizer s;
  TilePlan p;
  plan_carve(s, n, p);
  return s.used;
}

// Sorted coordinates (and the permutation for a grid): thread i handles caller
// index i < n and the padding position i in [n, npad).
__global__ void plan_points_kernel(int n, int npad, const float* __restrict__ px, const float* __restrict__ py, int m,
                                   int* perm, float* xs, float* ys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  if (i >= n) {
    xs[i] = 0.f;
    ys[i] = 0.f;
    if (perm) perm[i] = -1;
    return;
  }
  int r = i;
  if (m > 0) {
    const int fy = i / m, fx = i - fy * m;
    r = zorder_rank(fx, fy, m);
    perm[r] = i;
  }
  xs[r] = px[i];
  ys[r] = py[i];
}

// Bounding box of each chunk of 32 sorted points (valid points only). A chunk
// holding a non-finite coordinate gets an infinite box so it is never dropped.
__global__ void plan_boxes_kernel(int n, int nch, const float* __restrict__ xs, const float* __restrict__ ys,
                                  float4* cbox) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nch) return;
  float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  bool bad = false;
  const int jend = min(n, (c + 1) * kChunk);
  for (int j = c * kChunk; j < jend; ++j) {
    const float x = xs[j], y = ys[j];
    bad |= !(isfinite(x) && isfinite(y));
    x0 = fminf(x0, x);
    x1 = fmaxf(x1, x);
    y0 = fminf(y0, y);
    y1 = fmaxf(y1, y);
  }
  cbox[c] = bad ? make_float4(-INFINITY, INFINITY, -INFINITY, INFINITY) : make_float4(x0, x1, y0, y1);
}

// One wave per row tile: ascending list of live chunks by ballot compaction.
__global__ __launch_bounds__(64) void plan_lists_kernel(int nrt, int nch, const float4* __restrict__ cbox, float s2,
                                                        float threshold, int* count, int* nseg, uint16_t* list) {
  const int r = blockIdx.x;
  if (r >= nrt) return;
  const int lane = threadIdx.x;
  const float4 a = cbox[2 * r], b = cbox[2 * r + 1];
  const float rx0 = fminf(a.x, b.x), rx1 = fmaxf(a.y, b.y), ry0 = fminf(a.z, b.z), ry1 = fmaxf(a.w, b.w);
  uint16_t* out = list + (size_t)r * nch;
  int base = 0;
  for (int c0 = 0; c0 < nch; c0 += 64) {
    const int c = c0 + lane;
    bool live = false;
    if (c < nch) {
      const float4 q = cbox[c];
      const float gx = fmaxf(0.f, fmaxf(q.x - rx1, rx0 - q.y));
      const float gy = fmaxf(0.f, fmaxf(q.z - ry1, ry0 - q.w));
      live = !(s2 * fmaf(gx, gx, gy * gy) >= threshold);
    }
    const unsigned long long mask = __ballot(live);
    if (live) out[base + __popcll(mask & ((1ull << lane) - 1ull))] = (uint16_t)c;
    base += __popcll(mask);
  }
  if (lane == 0) {
    count[r] = base;
    nseg[r] = min(kMaxSeg, max(1, cdiv(base, kSegChunks)));
  }
}

int plan_build(TilePlan& p, int n, const float* px, const float* py, const gpl_grid* grid, float s2, float threshold,
               hipStream_t stream) {
  GPL_REQUIRE(n >= 1, "plan needs at least one point");
  GPL_REQUIRE(p.nch <= kMaxPlanChunks, "n=%d exceeds the product's limit of %d points", n, kMaxPlanChunks * kChunk);
  int m = 0;
  if (grid) {
    m = grid->n * grid->ss;
    GPL_REQUIRE(m > 0 && (long)m * m == n, "grid does not match n=%d", n);
  }
  int* perm = const_cast<int*>(p.perm);
  if (!grid) p.perm = nullptr;
  hipLaunchKernelGGL(plan_points_kernel, dim3(cdiv(p.npad, 256)), dim3(256), 0, stream, n, p.npad, px, py, m,
                     grid ? perm : nullptr, p.xs, p.ys);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_boxes_kernel, dim3(cdiv(p.nch, 256)), dim3(256), 0, stream, n, p.nch, p.xs, p.ys, p.cbox);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_lists_kernel, dim3(p.nrt), dim3(64), 0, stream, p.nrt, p.nch, p.cbox, s2, threshold,
                     p.count, p.nseg, p.list);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl
