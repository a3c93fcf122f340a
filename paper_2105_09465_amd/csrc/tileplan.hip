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
                                                        float threshold, int* count, uint16_t* list) {
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
  if (lane == 0) count[r] = base;
}

// Exclusive prefix sum of n ints in one workgroup of 1024 threads (in place
// allowed); the sum goes to *sum.
__global__ __launch_bounds__(1024) void plan_scan_kernel(int n, const int* in, int* out, int* sum) {
  __shared__ int wsum[16];
  __shared__ int carry_s;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int i = base + tid;
    const int v = i < n ? in[i] : 0;
    int x = v;  // inclusive scan within the wave
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int before = carry_s;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    if (i < n) out[i] = before + x - v;
    __syncthreads();
    if (tid == 1023) carry_s = before + x;
    __syncthreads();
  }
  if (tid == 0) *sum = carry_s;
}

// Largest row tile r with unit_off[r] <= u.
__device__ __forceinline__ int row_of_unit(const int* unit_off, int nrt, int u) {
  int lo = 0, hi = nrt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (unit_off[mid] <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Largest wave w with wave_unit(w) <= u (the wave whose range holds unit u).
__device__ __forceinline__ int wave_of_unit(int u, int T, int nw) {
  int lo = 0, hi = nw - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wave_unit(mid, T, nw) <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Per wave: first row tile and number of row tiles its units touch (the count
// goes to nrows[w], scanned into partial slots afterwards).
__global__ void plan_waves_kernel(int nrt, int nw, const int* unit_off, const int* total, int* wrow, int* nrows) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const int T = *total;
  const int u0 = wave_unit(w, T, nw), u1 = wave_unit(w + 1, T, nw);
  if (u0 >= u1) {
    wrow[w] = -1;
    nrows[w] = 0;
    return;
  }
  const int r0 = row_of_unit(unit_off, nrt, u0), r1 = row_of_unit(unit_off, nrt, u1 - 1);
  wrow[w] = r0;
  nrows[w] = r1 - r0 + 1;
}

// Per row tile: its partial slots [s0, s0 + cnt), from the first and last wave
// holding its units (waves in between start in this row tile, so their slots
// for it are their first ones, and empty waves own no slot).
__global__ void plan_rowslots_kernel(int nrt, int nw, const int* unit_off, const int* count, const int* total,
                                     const int* wrow, const int* wslot, int2* rslot) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrt) return;
  const int T = *total;
  const int a = unit_off[r], c = count[r];
  if (c <= 0) {
    rslot[r] = make_int2(0, 0);
    return;
  }
  const int wf = wave_of_unit(a, T, nw), wl = wave_of_unit(a + c - 1, T, nw);
  const int s0 = wslot[wf] + (r - wrow[wf]);
  const int s1 = wslot[wl] + (r - wrow[wl]);
  rslot[r] = make_int2(s0, s1 - s0 + 1);
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
  if (!grid) p.perm = nullptr;  // identity: the buffer stays unused
  hipLaunchKernelGGL(plan_points_kernel, dim3(cdiv(p.npad, 256)), dim3(256), 0, stream, n, p.npad, px, py, m,
                     grid ? perm : nullptr, p.xs, p.ys);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_boxes_kernel, dim3(cdiv(p.nch, 256)), dim3(256), 0, stream, n, p.nch, p.xs, p.ys, p.cbox);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_lists_kernel, dim3(p.nrt), dim3(64), 0, stream, p.nrt, p.nch, p.cbox, s2, threshold,
                     p.count, p.list);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_scan_kernel, dim3(1), dim3(1024), 0, stream, p.nrt, p.count, p.unit_off, p.total);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_waves_kernel, dim3(cdiv(p.nw, 256)), dim3(256), 0, stream, p.nrt, p.nw, p.unit_off, p.total,
                     p.wrow, p.wslot);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_scan_kernel, dim3(1), dim3(1024), 0, stream, p.nw, p.wslot, p.wslot, p.wslot + p.nw);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_rowslots_kernel, dim3(cdiv(p.nrt, 256)), dim3(256), 0, stream, p.nrt, p.nw, p.unit_off,
                     p.count, p.total, p.wrow, p.wslot, p.rslot);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl
