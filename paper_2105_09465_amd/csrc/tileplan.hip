// Construction of the tile plan of the kernel product (see tileplan.hpp): sorted
// points, chunk bounding boxes, and per row tile the list of chunks within the
// exact-zero cutoff of the kernel (Sec. 3.1, eq. "grbf").
#include <cmath>
#include <utility>

#include "tileplan.hpp"

namespace gpl {

size_t plan_workspace(int n) {
  if (n <= 0) return 0;
  Sizer s;
  TilePlan p;
  plan_carve(s, n, p);
  return s.used;
}

// ---- point order: Hilbert keys, then a stable LSD radix sort ----

// Extent of the finite points (one workgroup): (xmin, ymin, side of the square
// from there that holds them all, 0).
__global__ __launch_bounds__(1024) void plan_extent_kernel(int n, const float* __restrict__ px,
                                                           const float* __restrict__ py, float4* ext) {
  __shared__ float red[4][16];
  float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  // 8 points per thread and round, their loads issued together (an index past n
  // reads point 0 and is not used)
  constexpr int kU = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += kU * blockDim.x) {
    float x[kU], y[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * blockDim.x;
      x[u] = px[i < n ? i : 0];
      y[u] = py[i < n ? i : 0];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (i0 + u * (int)blockDim.x >= n || !(isfinite(x[u]) && isfinite(y[u]))) continue;
      x0 = fminf(x0, x[u]);
      x1 = fmaxf(x1, x[u]);
      y0 = fminf(y0, y[u]);
      y1 = fmaxf(y1, y[u]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    x0 = fminf(x0, __shfl_xor(x0, off, 64));
    x1 = fmaxf(x1, __shfl_xor(x1, off, 64));
    y0 = fminf(y0, __shfl_xor(y0, off, 64));
    y1 = fmaxf(y1, __shfl_xor(y1, off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = x0;
    red[1][w] = x1;
    red[2][w] = y0;
    red[3][w] = y1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      x0 = fminf(x0, red[0][k]);
      x1 = fmaxf(x1, red[1][k]);
      y0 = fminf(y0, red[2][k]);
      y1 = fmaxf(y1, red[3][k]);
    }
    if (!(x0 <= x1)) *ext = make_float4(0.f, 0.f, 0.f, 0.f);  // no finite point
    else *ext = make_float4(x0, y0, fmaxf(x1 - x0, y1 - y0), 0.f);
  }
}

// Index of cell (x, y) along the Hilbert curve of a 2^kHilbertBits square grid:
// at each level the quadrant contributes its position along the curve's U
// (0 lower left, 1 upper left, 2 upper right, 3 lower right), and the cell is
// mapped into the frame of that quadrant's copy of the curve.
__device__ __forceinline__ uint32_t hilbert_index(uint32_t x, uint32_t y) {
  constexpr uint32_t side = 1u << kHilbertBits;
  uint32_t d = 0;
  for (uint32_t s = side >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x ^= side - 1;
        y ^= side - 1;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

// Sort key of every point: its Hilbert index on the grid over the extent; a
// point with a non-finite coordinate takes the last key.
__global__ void plan_keys_kernel(int n, const float* __restrict__ px, const float* __restrict__ py,
                                 const float4* __restrict__ ext, uint32_t* __restrict__ key) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 e = *ext;
  const float x = px[i], y = py[i];
  constexpr float kMaxCell = (float)((1u << kHilbertBits) - 1);
  uint32_t k = (1u << (2 * kHilbertBits)) - 1;
  if (isfinite(x) && isfinite(y)) {
    const float sc = e.z > 0.f ? (float)(1u << kHilbertBits) / e.z : 0.f;
    const float qx = fminf(fmaxf((x - e.x) * sc, 0.f), kMaxCell);
    const float qy = fminf(fmaxf((y - e.y) * sc, 0.f), kMaxCell);
    k = hilbert_index((uint32_t)qx, (uint32_t)qy);
  }
  key[i] = k;
}

// Digit counts of one radix pass: hist[d nsb + b] = points of sort block b with
// digit d.
__global__ __launch_bounds__(kSortBlock) void sort_count_kernel(int n, int nsb, int shift,
                                                                const uint32_t* __restrict__ key,
                                                                int* __restrict__ hist) {
  __shared__ int h[kSortDigits];
  for (int d = threadIdx.x; d < kSortDigits; d += kSortBlock) h[d] = 0;
  __syncthreads();
  const int e = blockIdx.x * kSortBlock + threadIdx.x;
  if (e < n) atomicAdd(&h[(key[e] >> shift) & (kSortDigits - 1)], 1);
  __syncthreads();
  for (int d = threadIdx.x; d < kSortDigits; d += kSortBlock) hist[d * nsb + blockIdx.x] = h[d];
}

// Stable scatter of one radix pass. hist holds the exclusive scan of the counts
// (digit-major), i.e. the first output position of each (digit, block). A
// point's position adds the points of its block before it with the same digit:
// those in earlier waves (per-wave digit counts in LDS) and those in lower lanes
// of its own wave (the lanes that agree with it on all 8 digit bits, from 8
// ballots). vin = nullptr stands for the identity.
__global__ __launch_bounds__(kSortBlock) void sort_scatter_kernel(int n, int nsb, int shift,
                                                                  const uint32_t* __restrict__ kin,
                                                                  const int* __restrict__ vin,
                                                                  const int* __restrict__ hist,
                                                                  uint32_t* __restrict__ kout,
                                                                  int* __restrict__ vout) {
  constexpr int kWaves = kSortBlock / 64;
  __shared__ int wc[kWaves][kSortDigits];
  for (int i = threadIdx.x; i < kWaves * kSortDigits; i += kSortBlock) (&wc[0][0])[i] = 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * kSortBlock + threadIdx.x;
  const bool valid = e < n;
  const uint32_t k = valid ? kin[e] : 0u;
  const int v = valid ? (vin ? vin[e] : e) : 0;
  const int d = (int)((k >> shift) & (kSortDigits - 1));
  unsigned long long m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1;
    const unsigned long long bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  const int lower = __popcll(m & ((1ull << lane) - 1ull));
  __syncthreads();  // counts cleared
  if (valid && lower == 0) wc[w][d] = __popcll(m);
  __syncthreads();
  if (!valid) return;
  int r = hist[d * nsb + blockIdx.x] + lower;
  for (int q = 0; q < w; ++q) r += wc[q][d];
  kout[r] = k;
  vout[r] = v;
}

// Sorted coordinates and both directions of the permutation: thread r handles
// sorted position r < n (caller index sorted[r]) and padding position r in
// [n, npad).
__global__ void plan_points_kernel(int n, int npad, const float* __restrict__ px, const float* __restrict__ py,
                                   const int* sorted, int* perm, int* __restrict__ irank, float* __restrict__ xs,
                                   float* __restrict__ ys) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= npad) return;
  if (r >= n) {
    xs[r] = 0.f;
    ys[r] = 0.f;
    perm[r] = -1;
    return;
  }
  const int i = sorted[r];
  if ((unsigned)i >= (unsigned)n) {  // not a permutation: leave a hole, never an out-of-range write
    xs[r] = ys[r] = NAN;
    perm[r] = -1;
    return;
  }
  perm[r] = i;
  irank[i] = r;
  xs[r] = px[i];
  ys[r] = py[i];
}

// Scaled, block-centred coordinates (TilePlan::xc, yc, cen): thread r handles
// sorted position r. The block centre is the middle of the block's box, scaled
// and rounded to a multiple of 2^-12 (a float), and xc = sqrt(s2) x - centre is
// formed in FP64 and rounded once.
__global__ void plan_scaled_kernel(int npad, const float* __restrict__ xs, const float* __restrict__ ys,
                                   const float4* __restrict__ cbox, float s2, float* __restrict__ xc,
                                   float* __restrict__ yc, float2* __restrict__ cen) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= npad) return;
  const int b = r / kRowTile;
  const double sg = sqrt((double)s2);
  const float4 u = cbox[kChunksPerTile * b], v = cbox[kChunksPerTile * b + 1];
  const double mx = 0.5 * ((double)fminf(u.x, v.x) + (double)fmaxf(u.y, v.y));
  const double my = 0.5 * ((double)fminf(u.z, v.z) + (double)fmaxf(u.w, v.w));
  const float cx = isfinite(mx) ? (float)(rint(mx * sg * 4096.0) / 4096.0) : 0.f;
  const float cy = isfinite(my) ? (float)(rint(my * sg * 4096.0) / 4096.0) : 0.f;
  xc[r] = (float)((double)xs[r] * sg - (double)cx);
  yc[r] = (float)((double)ys[r] * sg - (double)cy);
  if (r == b * kRowTile) cen[b] = make_float2(cx, cy);
}

// Bounding box of the valid points in [j0, j1); a non-finite coordinate gives
// an infinite box (never dropped), no valid point an empty one (always dropped).
__device__ __forceinline__ float4 point_box(const float* __restrict__ xs, const float* __restrict__ ys, int j0,
                                            int j1) {
  float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  bool bad = false;
  for (int j = j0; j < j1; ++j) {
    const float x = xs[j], y = ys[j];
    bad |= !(isfinite(x) && isfinite(y));
    x0 = fminf(x0, x);
    x1 = fmaxf(x1, x);
    y0 = fminf(y0, y);
    y1 = fmaxf(y1, y);
  }
  return bad ? make_float4(-INFINITY, INFINITY, -INFINITY, INFINITY) : make_float4(x0, x1, y0, y1);
}

// Boxes of each chunk of 32 sorted points and of its two 16-point subtiles.
__global__ void plan_boxes_kernel(int n, int nch, const float* __restrict__ xs, const float* __restrict__ ys,
                                  float4* cbox, float4* sbox) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nch) return;
  const int j0 = c * kChunk, jm = min(n, j0 + kSubTile), j1 = min(n, j0 + kChunk);
  const float4 a = point_box(xs, ys, j0, jm), b = point_box(xs, ys, jm, j1);
  sbox[2 * c] = a;
  sbox[2 * c + 1] = b;
  cbox[c] = make_float4(fminf(a.x, b.x), fmaxf(a.y, b.y), fminf(a.z, b.z), fmaxf(a.w, b.w));
}

// One wave per row tile: ascending list of live chunks by ballot compaction,
// each entry with the mask of the subtiles that see the chunk and the mask of
// those that also need the lo part (gap below lo_threshold).
__global__ __launch_bounds__(64) void plan_lists_kernel(int nrt, int nch, const float4* __restrict__ cbox,
                                                        const float4* __restrict__ sbox, float s2, float threshold,
                                                        float lo_threshold, int* count, uint32_t* list, int* roww) {
  const int r = blockIdx.x;
  if (r >= nrt) return;
  const int lane = threadIdx.x;
  float4 sb[kSubsPerTile];
#pragma unroll
  for (int t = 0; t < kSubsPerTile; ++t) sb[t] = sbox[kSubsPerTile * r + t];
  float4 rb = cbox[kChunksPerTile * r];
#pragma unroll
  for (int t = 1; t < kChunksPerTile; ++t) {
    const float4 c = cbox[kChunksPerTile * r + t];
    rb = make_float4(fminf(rb.x, c.x), fmaxf(rb.y, c.y), fminf(rb.z, c.z), fmaxf(rb.w, c.w));
  }
  uint32_t* out = list + (size_t)r * nch;
  int base = 0, cost = 0;
  for (int c0 = 0; c0 < nch; c0 += 64) {
    const int c = c0 + lane;
    unsigned mask = 0u;
    if (c < nch) {
      const float4 q = cbox[c];
      if (boxes_live(rb, q, s2, threshold)) {
#pragma unroll
        for (int t = 0; t < kSubsPerTile; ++t) {
          mask |= (boxes_live(sb[t], q, s2, threshold) ? 1u : 0u) << t;
          mask |= (boxes_live(sb[t], q, s2, lo_threshold) ? 1u : 0u) << (4 + t);
        }
      }
    }
    const bool live = (mask & 0xfu) != 0u;
    const unsigned long long bal = __ballot(live);
    const uint32_t e = (uint32_t)c | (mask << 16);
    if (live) {
      out[base + __popcll(bal & ((1ull << lane) - 1ull))] = e;
      cost += unit_cost(e);
    }
    base += __popcll(bal);
  }
  for (int off = 32; off > 0; off >>= 1) cost += __shfl_xor(cost, off, 64);
  if (lane == 0) {
    count[r] = base;
    roww[r] = kCostRowTile + cost;
  }
}

// Exclusive prefix sum of n ints in one workgroup of 1024 threads (in place
// allowed); the sum goes to *sum. A round covers 16384 entries: they are loaded
// into LDS with coalesced loads, each thread scans 16 consecutive ones (row
// stride 17 words, so the 64 lanes of a wave hit distinct banks), the thread
// totals are scanned across the workgroup, and the results go back through LDS
// to coalesced stores. T (the output type) is int or long long.
constexpr int kScanIpt = 16;
constexpr int kScanRound = 1024 * kScanIpt;
template <class T>
__global__ __launch_bounds__(1024) void plan_scan_kernel(int n, const int* in, T* out, T* sum) {
  __shared__ T buf[1024 * (kScanIpt + 1)];
  __shared__ T wsum[16];
  __shared__ T carry_s;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) carry_s = 0;
  for (int base = 0; base < n; base += kScanRound) {
    __syncthreads();  // the previous round's stores have read buf
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
      const int e = k * 1024 + tid;  // entry of the round, coalesced
      buf[(e / kScanIpt) * (kScanIpt + 1) + e % kScanIpt] = base + e < n ? (T)in[base + e] : (T)0;
    }
    __syncthreads();
    T* row = buf + tid * (kScanIpt + 1);
    T tot = 0;
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) tot += row[k];
    T x = tot;  // inclusive scan of the thread totals within the wave
    for (int off = 1; off < 64; off <<= 1) {
      const T y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    T before = carry_s;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    T run = before + x - tot;
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
      const T v = row[k];
      row[k] = run;
      run += v;
    }
    __syncthreads();
    if (tid == 1023) carry_s = before + x;
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
      const int e = k * 1024 + tid;
      if (base + e < n) out[base + e] = buf[(e / kScanIpt) * (kScanIpt + 1) + e % kScanIpt];
    }
  }
  __syncthreads();
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

// Largest wave w with wunit[w] <= u (the wave whose range holds unit u).
__device__ __forceinline__ int wave_of_unit(int u, const int* wunit, int nw) {
  int lo = 0, hi = nw - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wunit[mid] <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// First unit of each wave b in [0, nw]: the first unit whose exclusive cost
// prefix reaches the wave's target, wtot x (round weight of the waves below b)
// / (that of all nw waves). A row tile's own cost counts before its first unit.
// One wave per boundary: the row tile by binary search over the row prefixes,
// then the units of that row tile 64 at a time.
__global__ __launch_bounds__(256) void plan_wunit_kernel(int nrt, int nch, int nw, int wround, const int* count,
                                                         const uint32_t* __restrict__ list, const int* unit_off,
                                                         const long long* rowwoff, const long long* wtot, int* wunit) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b > nw) return;
  const long long t = *wtot * wave_weight_below(b, wround) / wave_weight_below(nw, wround);
  int lo = 0, hi = nrt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rowwoff[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int r = lo, cnt = count[r];
  const long long rem = t - rowwoff[r];
  const uint32_t* L = list + (size_t)r * nch;
  long long before = kCostRowTile;  // cost of the row tile up to the current group of 64 units
  int k = 0;
  for (int k0 = 0; k0 < cnt && before < rem; k0 += 64) {
    const int kk = k0 + lane;
    const int c = kk < cnt ? unit_cost(L[kk]) : 0;
    int x = c;  // inclusive prefix within the group
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    k += __popcll(__ballot(kk < cnt && before + (x - c) < rem));
    before += __shfl(x, 63, 64);
  }
  if (lane == 0) wunit[b] = unit_off[r] + k;
}

// Per wave: first row tile and number of row tiles its units touch (the count
// goes to nrows[w], scanned into partial slots afterwards).
__global__ void plan_waves_kernel(int nrt, int nw, const int* wunit, const int* unit_off, int* wrow, int* nrows) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const int u0 = wunit[w], u1 = wunit[w + 1];
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
__global__ void plan_rowslots_kernel(int nrt, int nw, const int* wunit, const int* unit_off, const int* count,
                                     const int* wrow, const int* wslot, int2* rslot) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrt) return;
  const int a = unit_off[r], c = count[r];
  if (c <= 0) {
    rslot[r] = make_int2(0, 0);
    return;
  }
  const int wf = wave_of_unit(a, wunit, nw), wl = wave_of_unit(a + c - 1, wunit, nw);
  const int s0 = wslot[wf] + (r - wrow[wf]);
  const int s1 = wslot[wl] + (r - wrow[wl]);
  rslot[r] = make_int2(s0, s1 - s0 + 1);
}

// Per wave, its range in one load: the first row tile r, its first partial
// slot, the list positions [kb, ke) it takes in row tile r, and the number of
// units it takes in the row tiles after r (-1 row tile: no units).
__global__ void plan_wdesc_kernel(int nw, const int* wunit, const int* unit_off, const int* count, const int* wrow,
                                  const int* wslot, int4* wdesc, int* wrest) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const int u0 = wunit[w], u1 = wunit[w + 1];
  const int r = wrow[w];
  if (u0 >= u1 || r < 0) {
    wdesc[w] = make_int4(-1, wslot[w], 0, 0);
    wrest[w] = 0;
    return;
  }
  const int off = unit_off[r];
  const int ke = min(u1, off + count[r]) - off;
  wdesc[w] = make_int4(r, wslot[w], u0 - off, ke);
  wrest[w] = u1 - (off + ke);
}

// Compute units of the current device (queried once per device).
static int compute_units() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] <= 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}

int plan_sort(TilePlan& p, int n, const float* px, const float* py, hipStream_t stream) {
  GPL_REQUIRE(n >= 1, "plan needs at least one point");
  GPL_REQUIRE(p.nch <= kMaxPlanChunks, "n=%d exceeds the product's limit of %d points", n, kMaxPlanChunks * kChunk);
  int* perm = const_cast<int*>(p.perm);
  int* irank = const_cast<int*>(p.irank);
  const int nsb = sort_blocks(n);
  // sort scratch in buffers that are written only after the sort: the extent in
  // cbox[0], the keys in xc and yc, the scan totals in total
  float4* ext = p.cbox;
  hipLaunchKernelGGL(plan_extent_kernel, dim3(1), dim3(1024), 0, stream, n, px, py, ext);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_keys_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, px, py, ext,
                     reinterpret_cast<uint32_t*>(p.xc));
  GPL_LAUNCH_CHECK();
  // ping-pong: keys xc <-> yc, caller indices (identity) -> sval <-> perm
  uint32_t* kin = reinterpret_cast<uint32_t*>(p.xc);
  uint32_t* kout = reinterpret_cast<uint32_t*>(p.yc);
  const int* vin = nullptr;
  int* vout = p.sval;
  for (int pass = 0; pass < kSortPasses; ++pass) {
    hipLaunchKernelGGL(sort_count_kernel, dim3(nsb), dim3(kSortBlock), 0, stream, n, nsb, 8 * pass, kin, p.shist);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(plan_scan_kernel<int>, dim3(1), dim3(1024), 0, stream, kSortDigits * nsb, p.shist, p.shist,
                       p.total);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(sort_scatter_kernel, dim3(nsb), dim3(kSortBlock), 0, stream, n, nsb, 8 * pass, kin, vin,
                       p.shist, kout, vout);
    GPL_LAUNCH_CHECK();
    std::swap(kin, kout);
    vin = vout;
    vout = vout == p.sval ? perm : p.sval;
  }
  hipLaunchKernelGGL(plan_points_kernel, dim3(cdiv(p.npad, 256)), dim3(256), 0, stream, n, p.npad, px, py, vin, perm,
                     irank, p.xs, p.ys);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_boxes_kernel, dim3(cdiv(p.nch, 256)), dim3(256), 0, stream, n, p.nch, p.xs, p.ys, p.cbox,
                     p.sbox);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int plan_build(TilePlan& p, int n, const float* px, const float* py, const gpl_grid* grid, float s2, float threshold,
               float lo_threshold, hipStream_t stream) {
  if (grid) {
    const int m = grid->n * grid->ss;
    GPL_REQUIRE(m > 0 && (long)m * m == n, "grid does not match n=%d", n);
  }
  p.wround = 4 * compute_units();
  GPL_TRY(plan_sort(p, n, px, py, stream));
  hipLaunchKernelGGL(plan_scaled_kernel, dim3(cdiv(p.npad, 256)), dim3(256), 0, stream, p.npad, p.xs, p.ys, p.cbox, s2,
                     p.xc, p.yc, p.cen);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_lists_kernel, dim3(p.nrt), dim3(64), 0, stream, p.nrt, p.nch, p.cbox, p.sbox, s2,
                     threshold, lo_threshold, p.count, p.list, p.roww);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_scan_kernel<int>, dim3(1), dim3(1024), 0, stream, p.nrt, p.count, p.unit_off, p.total);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_scan_kernel<long long>, dim3(1), dim3(1024), 0, stream, p.nrt, p.roww, p.rowwoff, p.wtot);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_wunit_kernel, dim3(cdiv(p.nw + 1, 4)), dim3(256), 0, stream, p.nrt, p.nch, p.nw, p.wround,
                     p.count, p.list, p.unit_off, p.rowwoff, p.wtot, p.wunit);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_waves_kernel, dim3(cdiv(p.nw, 256)), dim3(256), 0, stream, p.nrt, p.nw, p.wunit,
                     p.unit_off, p.wrow, p.wslot);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_scan_kernel<int>, dim3(1), dim3(1024), 0, stream, p.nw, p.wslot, p.wslot, p.wslot + p.nw);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_rowslots_kernel, dim3(cdiv(p.nrt, 256)), dim3(256), 0, stream, p.nrt, p.nw, p.wunit,
                     p.unit_off, p.count, p.wrow, p.wslot, p.rslot);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(plan_wdesc_kernel, dim3(cdiv(p.nw, 256)), dim3(256), 0, stream, p.nw, p.wunit, p.unit_off,
                     p.count, p.wrow, p.wslot, p.wdesc, p.wrest);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl
