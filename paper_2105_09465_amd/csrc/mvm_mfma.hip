// Kernel-matrix product on MFMA: Y = K V + beta Y with K_ij = a^2 exp(-|p_i-p_j|^2/(2 l^2))
// (eq. "grbf"), the exp tile formed in registers and contracted with the
// right-hand-side block on the matrix cores (the tile x RHS product is a true
// dense contraction). K is never stored (Sec. 3.3).
//
// Work decomposition: the points are taken in the order of a tile plan
// (tileplan.hpp), which lists for every row tile of 64 points the chunks of 32
// points that can give a non-zero kernel value; every other pair contributes
// exact zeros and is not evaluated. A work item is one row tile and one
// contiguous segment of its chunk list; its workgroup of 4 waves computes the
// same 64 rows (four 16-row MFMA tiles per wave) over interleaved chunks, with
// the chunk's coordinates and right-hand-side block loaded straight from global
// memory into the MFMA B-operand layout, and sums the 4 waves' accumulators in
// LDS in a fixed order. Items write partial rows; a reduction kernel adds the
// items of each row tile in order and scatters to the caller's order, so the
// result is bitwise reproducible. Exact coordinate differences are formed
// before scaling.
//
// Precision form (GPL_PREC_F16X3): exp tiles computed in FP32 as 2^11 k (the
// factor enters through the exp2 argument) and split into FP16 hi (the top 11
// significant bits) and lo = k - hi; the RHS block is split the same way after
// a per-column power-of-two scale that puts its largest entry near 2^14. Each
// 16x16x32 tile takes three MFMAs (hi.hi + hi.lo + lo.hi) into FP32
// accumulators; the dropped lo.lo term is ~2^-22 relative.
//
// FP32 form (GPL_PREC_FP32): the exp tile and the RHS in FP32 on
// v_mfma_f32_16x16x4_f32.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"
#include "mvm_mfma.hpp"
#include "timing.hpp"

namespace gpl {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRT = 4;                      // 16-row MFMA tiles per wave
constexpr int kWaves = 4;                   // waves per workgroup (one work item)
constexpr float kKScale = 2048.f;           // 2^11 applied to the FP16 exp tile
static constexpr int kMaxCB = 4;            // up to 64 columns per pass

static_assert(kRT * 16 == kRowTile, "row tile is four MFMA tiles");

// ---------------------------------------------------------------- RHS preparation

// Column-wise max |V| in two steps without atomics: kColmaxBlocks workgroups per
// column write partial maxima (as bit patterns of non-negative floats); the
// split kernel folds them.
__device__ __forceinline__ void colmax_body(int bx, int c, int n, const float* __restrict__ V, int ldv,
                                            unsigned* partial) {
  __shared__ float red[4];
  float m = 0.f;
  for (int i = bx * blockDim.x + threadIdx.x; i < n; i += kColmaxBlocks * blockDim.x)
    m = fmaxf(m, fabsf(V[(size_t)c * ldv + i]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[c * kColmaxBlocks + bx] = __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
}

__global__ __launch_bounds__(256) void colmax_kernel(int n, const float* __restrict__ V, int ldv, unsigned* partial,
                                                     CgGate gate) {
  if (gate.skip_all()) return;
  colmax_body(blockIdx.x, blockIdx.y, n, V, ldv, partial);
}

// Sorted position j of column c: the caller's row perm[j] (or j), zero past n
// and for c >= nrhs.
__device__ __forceinline__ float gather_rhs(int j, int c, int n, int nrhs, const int* perm, const float* V, int ldv) {
  if (c >= nrhs || j >= n) return 0.f;
  return V[(size_t)c * ldv + (perm ? perm[j] : j)];
}

// V' = V * 2^e_c split into FP16 hi (nearest) and lo, in sorted order;
// inv_scale[c] = 2^-e_c / 2^11 folds both scales for the output.
__device__ __forceinline__ void split_rhs_body(int bx, int c, int n, int nrhs, const float* __restrict__ V, int ldv,
                                               const int* perm, const unsigned* colmax, _Float16* Vh, _Float16* Vl,
                                               int ldh, float* inv_scale) {
  const int j = bx * blockDim.x + threadIdx.x;
  if (j >= ldh) return;
  int e = 0;
  if (c < nrhs) {
    unsigned mb = 0u;
    for (int b = 0; b < kColmaxBlocks; ++b) mb = max(mb, colmax[c * kColmaxBlocks + b]);
    const float mx = __uint_as_float(mb);
    if (mx > 0.f && isfinite(mx)) e = 14 - ilogbf(mx) - 1;  // mx * 2^e in [2^13, 2^14)
  }
  const float scale = ldexpf(1.f, e);
  if (j == 0) inv_scale[c] = ldexpf(1.f, -e) / kKScale;
  const float v = gather_rhs(j, c, n, nrhs, perm, V, ldv) * scale;
  const _Float16 h = (_Float16)v;
  const _Float16 l = (_Float16)(v - (float)h);
  Vh[(size_t)c * ldh + j] = h;
  Vl[(size_t)c * ldh + j] = l;
}

__global__ void split_rhs_kernel(int n, int nrhs, const float* __restrict__ V, int ldv, const int* perm,
                                 const unsigned* colmax, _Float16* Vh, _Float16* Vl, int ldh, float* inv_scale,
                                 CgGate gate) {
  if (gate.skip_all()) return;
  split_rhs_body(blockIdx.x, blockIdx.y, n, nrhs, V, ldv, perm, colmax, Vh, Vl, ldh, inv_scale);
}

// FP32 form: the RHS block in sorted order, zero padded.
__device__ __forceinline__ void pack_rhs_body(int bx, int c, int n, int nrhs, const float* __restrict__ V, int ldv,
                                              const int* perm, float* Vp, int ldh) {
  const int j = bx * blockDim.x + threadIdx.x;
  if (j >= ldh) return;
  Vp[(size_t)c * ldh + j] = gather_rhs(j, c, n, nrhs, perm, V, ldv);
}

__global__ void pack_rhs_kernel(int n, int nrhs, const float* __restrict__ V, int ldv, const int* perm, float* Vp,
                                int ldh, CgGate gate) {
  if (gate.skip_all()) return;
  pack_rhs_body(blockIdx.x, blockIdx.y, n, nrhs, V, ldv, perm, Vp, ldh);
}

// ---------------------------------------------------------------- work items

struct Item {
  int r, beg, end;
};

// Work item `item` of a plan: row tile item / kMaxSeg and its segment of the
// chunk list (r = -1 when the item is unused).
__device__ __forceinline__ Item item_of(int item, const TilePlan& P) {
  Item it{-1, 0, 0};
  const int r = item / kMaxSeg, s = item - r * kMaxSeg;
  if (r >= P.nrt) return it;
  const int ns = P.nseg[r];
  if (s >= ns) return it;
  const int L = P.count[r];
  it.r = r;
  it.beg = L * s / ns;  // L < 2^16, s < kMaxSeg: no overflow
  it.end = L * (s + 1) / ns;
  return it;
}

// Chunk k of a row tile's list, read through the scalar unit (k is uniform per
// wave; rows of the list start 4-byte aligned since nch is even).
__device__ __forceinline__ int chunk_at(const uint16_t* lst, int k) {
  const uint32_t w = reinterpret_cast<const uint32_t*>(lst)[k >> 1];
  return (int)((k & 1) ? (w >> 16) : (w & 0xffffu));
}

// Fixed-order sum of the 4 waves' accumulators of a work item and the write of
// its partial rows: part[(item * pcols + c0 + c) * 64 + row] for c < ncols.
template <int CB>
__device__ __forceinline__ void item_store(f32x4 (&acc)[kRT][CB], int item, float* __restrict__ part, int pcols,
                                           int c0, int ncols) {
  __shared__ f32x4 red[kWaves - 1][kRT * CB][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave > 0) {
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) red[wave - 1][rt * CB + cb][lane] = acc[rt][cb];
  }
  __syncthreads();
  if (wave != 0) return;
  const int ri = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      f32x4 s = acc[rt][cb];
#pragma unroll
      for (int w = 0; w < kWaves - 1; ++w) s += red[w][rt * CB + cb][lane];
      const int c = cb * 16 + ri;  // D layout: column = lane % 16, rows 4 * (lane / 16) + v
      if (c < ncols)
        *reinterpret_cast<f32x4*>(&part[((size_t)item * pcols + c0 + c) * kRowTile + rt * 16 + g * 4]) = s;
    }
}

// ---------------------------------------------------------------- precision form

// Operands of one chunk for one lane: its 8 consecutive source points and the
// hi/lo RHS fragments of every column block (columns past nrhs are zero).
template <int CB>
struct F16Chunk {
  f32x4 x0, x1, y0, y1;
  half8 bh[CB], bl[CB];
};

template <int CB>
__device__ __forceinline__ void f16_load(F16Chunk<CB>& c, const TilePlan& P, const _Float16* __restrict__ Vh,
                                         const _Float16* __restrict__ Vl, int ldh, int ch, int ri, int g) {
  const int j0 = ch * kChunk + g * 8;
  c.x0 = *reinterpret_cast<const f32x4*>(&P.xs[j0]);
  c.x1 = *reinterpret_cast<const f32x4*>(&P.xs[j0 + 4]);
  c.y0 = *reinterpret_cast<const f32x4*>(&P.ys[j0]);
  c.y1 = *reinterpret_cast<const f32x4*>(&P.ys[j0 + 4]);
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const size_t o = (size_t)(cb * 16 + ri) * ldh + j0;
    c.bh[cb] = *reinterpret_cast<const half8*>(&Vh[o]);
    c.bl[cb] = *reinterpret_cast<const half8*>(&Vl[o]);
  }
}

template <int CB>
__device__ __forceinline__ void f16_compute(f32x4 (&acc)[kRT][CB], const F16Chunk<CB>& c, const float (&xi)[kRT],
                                            const float (&yi)[kRT], float s2) {
  const float xj[8] = {c.x0[0], c.x0[1], c.x0[2], c.x0[3], c.x1[0], c.x1[1], c.x1[2], c.x1[3]};
  const float yj[8] = {c.y0[0], c.y0[1], c.y0[2], c.y0[3], c.y1[0], c.y1[1], c.y1[2], c.y1[3]};
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    float hf[8], lf[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float dx = xi[rt] - xj[e], dy = yi[rt] - yj[e];
      const float d2 = fmaf(dx, dx, dy * dy);
      const float k2 = exp2_fast(fmaf(d2, -s2, 11.f));             // 2^11 k
      hf[e] = __uint_as_float(__float_as_uint(k2) & 0xffffe000u);  // top 11 significant bits
      lf[e] = k2 - hf[e];
    }
    half8 hi, lo;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      const half2v h = __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(hf[e], hf[e + 1]));
      const half2v l = __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(lf[e], lf[e + 1]));
      hi[e] = h[0];
      hi[e + 1] = h[1];
      lo[e] = l[0];
      lo[e + 1] = l[1];
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
      acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, c.bh[cb], acc[rt][cb], 0, 0, 0);
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
      acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, c.bl[cb], acc[rt][cb], 0, 0, 0);
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
      acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo, c.bh[cb], acc[rt][cb], 0, 0, 0);
  }
}

template <int CB>
__device__ __forceinline__ void mvm_f16x3_item(int item, const TilePlan P, float s2, const _Float16* __restrict__ Vh,
                                               const _Float16* __restrict__ Vl, int ldh, int ncols,
                                               float* __restrict__ part, int pcols, int c0) {
  const Item it = item_of(item, P);
  if (it.r < 0) return;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ri = lane & 15, g = lane >> 4;
  float xi[kRT], yi[kRT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    const int i = it.r * kRowTile + rt * 16 + ri;
    xi[rt] = P.xs[i];
    yi[rt] = P.ys[i];
  }
  f32x4 acc[kRT][CB];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // This wave's chunks are list entries kw, kw + 4, ...; their indices are
  // read 64 at a time, one per lane, and broadcast with readlane.
  const uint16_t* lst = P.list + (size_t)it.r * P.nch;
  const int kw = it.beg + wave;
  const int nk = kw < it.end ? (it.end - kw + kWaves - 1) / kWaves : 0;
#pragma unroll 1
  for (int t0 = 0; t0 < nk; t0 += 64) {
    const int m = min(64, nk - t0);
    const int vidx = lane < m ? (int)lst[kw + kWaves * (t0 + lane)] : 0;
    // two operand buffers: the next chunk's loads are in flight while the
    // current one is computed (a load past the end repeats the last chunk)
    F16Chunk<CB> a, b;
    f16_load(a, P, Vh, Vl, ldh, __builtin_amdgcn_readlane(vidx, 0), ri, g);
#pragma unroll 1
    for (int t = 0; t < m; t += 2) {
      f16_load(b, P, Vh, Vl, ldh, __builtin_amdgcn_readlane(vidx, min(t + 1, m - 1)), ri, g);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the compute
      f16_compute(acc, a, xi, yi, s2);
      if (t + 1 >= m) break;
      f16_load(a, P, Vh, Vl, ldh, __builtin_amdgcn_readlane(vidx, min(t + 2, m - 1)), ri, g);
      __builtin_amdgcn_sched_barrier(0);
      f16_compute(acc, b, xi, yi, s2);
    }
  }
  item_store<CB>(acc, item, part, pcols, c0, ncols);
}

template <int CB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CB >= 3 ? 2 : 3))) void mvm_f16x3_kernel(const TilePlan P, float s2, const _Float16* __restrict__ Vh,
                                                        const _Float16* __restrict__ Vl, int ldh, int ncols,
                                                        float* __restrict__ part, int pcols, int c0, CgGate gate) {
  if (gate.skip_all()) return;
  mvm_f16x3_item<CB>(blockIdx.x, P, s2, Vh, Vl, ldh, ncols, part, pcols, c0);
}

// ---------------------------------------------------------------- FP32 form

template <int CB>
__device__ __forceinline__ void mvm_f32_item(int item, const TilePlan P, float s2, const float* __restrict__ Vp,
                                             int ldh, int ncols, float* __restrict__ part, int pcols, int c0) {
  const Item it = item_of(item, P);
  if (it.r < 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ri = lane & 15, g = lane >> 4;
  float xi[kRT], yi[kRT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    const int i = it.r * kRowTile + rt * 16 + ri;
    xi[rt] = P.xs[i];
    yi[rt] = P.ys[i];
  }
  f32x4 acc[kRT][CB];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* lst = P.list + (size_t)it.r * P.nch;
#pragma unroll 1
  for (int k = it.beg + wave; k < it.end; k += kWaves) {
    // two groups of 16 points; in each, this lane's 4 consecutive points
    const int jc = (int)lst[k] * kChunk + g * 4;
    float xj[8], yj[8];
    *reinterpret_cast<f32x4*>(&xj[0]) = *reinterpret_cast<const f32x4*>(&P.xs[jc]);
    *reinterpret_cast<f32x4*>(&xj[4]) = *reinterpret_cast<const f32x4*>(&P.xs[jc + 16]);
    *reinterpret_cast<f32x4*>(&yj[0]) = *reinterpret_cast<const f32x4*>(&P.ys[jc]);
    *reinterpret_cast<f32x4*>(&yj[4]) = *reinterpret_cast<const f32x4*>(&P.ys[jc + 16]);
    f32x4 b[CB][2];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int c = cb * 16 + ri;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        b[cb][h] = c < ncols ? *reinterpret_cast<const f32x4*>(&Vp[(size_t)c * ldh + jc + 16 * h])
                             : f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      float kv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float dx = xi[rt] - xj[e], dy = yi[rt] - yj[e];
        const float d2 = fmaf(dx, dx, dy * dy);
        kv[e] = exp2_fast(-(d2 * s2));
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[e], b[cb][e >> 2][e & 3], acc[rt][cb], 0, 0, 0);
    }
  }
  item_store<CB>(acc, item, part, pcols, c0, ncols);
}

template <int CB>
__global__ __launch_bounds__(256) void mvm_f32_kernel(const TilePlan P, float s2, const float* __restrict__ Vp,
                                                      int ldh, int ncols, float* __restrict__ part, int pcols, int c0,
                                                      CgGate gate) {
  if (gate.skip_all()) return;
  mvm_f32_item<CB>(blockIdx.x, P, s2, Vp, ldh, ncols, part, pcols, c0);
}

// ---------------------------------------------------------------- reduction

// Y[c][perm[j]] = (amp2 * colscale[c]) * sum_s part[r, s][c][row] + beta Y, the
// items of row tile r = j / 64 in order.
__device__ __forceinline__ void reduce_body(int bx, int c, const TilePlan& P, int nrhs, const float* __restrict__ part,
                                            int pcols, const float* __restrict__ colscale, float amp2, float* Y,
                                            int ldy, float beta) {
  const int j = bx * blockDim.x + threadIdx.x;
  if (j >= P.n || c >= nrhs) return;
  const int r = j / kRowTile, row = j - r * kRowTile;
  const int ns = P.nseg[r];
  float s = 0.f;
  for (int q = 0; q < ns; ++q) s += part[((size_t)(r * kMaxSeg + q) * pcols + c) * kRowTile + row];
  const float f = colscale ? amp2 * colscale[c] : amp2;
  float* y = Y + (size_t)c * ldy + (P.perm ? P.perm[j] : j);
  const float res = f * s;
  *y = beta != 0.f ? res + beta * *y : res;
}

__global__ void reduce_kernel(const TilePlan P, int nrhs, const float* __restrict__ part, int pcols,
                              const float* __restrict__ colscale, float amp2, float* Y, int ldy, float beta,
                              CgGate gate) {
  if (gate.skip_all()) return;
  reduce_body(blockIdx.x, blockIdx.y, P, nrhs, part, pcols, colscale, amp2, Y, ldy, beta);
}

// ---------------------------------------------------------------- workspace

// Buffers of one product: RHS block in sorted order (FP16 hi/lo or FP32), the
// column scales and the partial rows of every work item.
struct ProdBufs {
  unsigned* colmax;
  float* inv_scale;
  _Float16 *Vh, *Vl;  // precision form
  float* Vp;          // FP32 form
  float* part;
  int ldh, ncp;
};

template <class C>
static void carve_prod(C& cv, int n, int nrhs, int prec, ProdBufs& b) {
  const int nrt = cdiv(n, kRowTile);
  b.ldh = nrt * kRowTile;
  b.ncp = cdiv(nrhs, 16) * 16;
  const bool f16 = prec == GPL_PREC_F16X3;
  b.colmax = f16 ? cv.template take<unsigned>((size_t)b.ncp * kColmaxBlocks) : nullptr;
  b.inv_scale = f16 ? cv.template take<float>(b.ncp) : nullptr;
  b.Vh = f16 ? cv.template take<_Float16>((size_t)b.ncp * b.ldh) : nullptr;
  b.Vl = f16 ? cv.template take<_Float16>((size_t)b.ncp * b.ldh) : nullptr;
  b.Vp = f16 ? nullptr : cv.template take<float>((size_t)b.ncp * b.ldh);
  b.part = cv.template take<float>((size_t)nrt * kMaxSeg * nrhs * kRowTile);
}

size_t mfma_workspace(int n, int nrhs, int prec) {
  if (n <= 0 || nrhs <= 0) return 0;
  Sizer s;
  ProdBufs b;
  carve_prod(s, n, nrhs, prec, b);
  return s.used;
}

float plan_threshold(int prec) { return prec == GPL_PREC_F16X3 ? kSkipF16x3 : kSkipFp32; }

// ---------------------------------------------------------------- launches

template <int CB>
static void launch_f16x3(const TilePlan& P, float s2, const _Float16* Vh, const _Float16* Vl, int ldh, int ncols,
                         float* part, int pcols, int c0, CgGate gate, hipStream_t stream) {
  hipLaunchKernelGGL((mvm_f16x3_kernel<CB>), dim3(P.nrt * kMaxSeg), dim3(256), 0, stream, P, s2, Vh, Vl, ldh, ncols,
                     part, pcols, c0, gate);
}

template <int CB>
static void launch_f32(const TilePlan& P, float s2, const float* Vp, int ldh, int ncols, float* part, int pcols,
                       int c0, CgGate gate, hipStream_t stream) {
  hipLaunchKernelGGL((mvm_f32_kernel<CB>), dim3(P.nrt * kMaxSeg), dim3(256), 0, stream, P, s2, Vp, ldh, ncols, part,
                     pcols, c0, gate);
}

int mfma_launch(const TilePlan& P, int prec, float s2, float amp2, int nrhs, const float* V, int ldv, float* Y,
                int ldy, float beta, void* ws, size_t ws_bytes, CgGate gate, hipStream_t stream) {
  const int n = P.n;
  GPL_TRY(check_ws(ws, ws_bytes, mfma_workspace(n, nrhs, prec)));
  Carver cv(ws, ws_bytes);
  ProdBufs b;
  carve_prod(cv, n, nrhs, prec, b);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  const bool f16 = prec == GPL_PREC_F16X3;
  if (f16) {
    hipLaunchKernelGGL(colmax_kernel, dim3(kColmaxBlocks, nrhs), dim3(256), 0, stream, n, V, ldv, b.colmax, gate);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(split_rhs_kernel, dim3(cdiv(b.ldh, 256), b.ncp), dim3(256), 0, stream, n, nrhs, V, ldv, P.perm,
                       b.colmax, b.Vh, b.Vl, b.ldh, b.inv_scale, gate);
  } else {
    hipLaunchKernelGGL(pack_rhs_kernel, dim3(cdiv(b.ldh, 256), b.ncp), dim3(256), 0, stream, n, nrhs, V, ldv, P.perm,
                       b.Vp, b.ldh, gate);
  }
  GPL_LAUNCH_CHECK();
  // column blocks of up to 64 columns per pass; each pass writes its own columns
  for (int c0 = 0; c0 < b.ncp; c0 += kMaxCB * 16) {
    const int cb = std::min(kMaxCB, (b.ncp - c0) / 16);
    const int ncols = std::min(nrhs - c0, cb * 16);
    hipEvent_t t0 = timing_begin(stream);
    if (f16) {
      const _Float16* vh = b.Vh + (size_t)c0 * b.ldh;
      const _Float16* vl = b.Vl + (size_t)c0 * b.ldh;
      switch (cb) {
        case 4: launch_f16x3<4>(P, s2, vh, vl, b.ldh, ncols, b.part, nrhs, c0, gate, stream); break;
        case 3: launch_f16x3<3>(P, s2, vh, vl, b.ldh, ncols, b.part, nrhs, c0, gate, stream); break;
        case 2: launch_f16x3<2>(P, s2, vh, vl, b.ldh, ncols, b.part, nrhs, c0, gate, stream); break;
        default: launch_f16x3<1>(P, s2, vh, vl, b.ldh, ncols, b.part, nrhs, c0, gate, stream); break;
      }
    } else {
      const float* vp = b.Vp + (size_t)c0 * b.ldh;
      switch (cb) {
        case 4: launch_f32<4>(P, s2, vp, b.ldh, ncols, b.part, nrhs, c0, gate, stream); break;
        case 3: launch_f32<3>(P, s2, vp, b.ldh, ncols, b.part, nrhs, c0, gate, stream); break;
        case 2: launch_f32<2>(P, s2, vp, b.ldh, ncols, b.part, nrhs, c0, gate, stream); break;
        default: launch_f32<1>(P, s2, vp, b.ldh, ncols, b.part, nrhs, c0, gate, stream); break;
      }
    }
    GPL_LAUNCH_CHECK();
    timing_end(t0, stream);
  }
  hipLaunchKernelGGL(reduce_kernel, dim3(cdiv(n, 256), nrhs), dim3(256), 0, stream, P, nrhs, b.part, nrhs,
                     f16 ? b.inv_scale : nullptr, amp2, Y, ldy, beta, gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

// ---------------------------------------------------------------- grouped launches (serving)
// One launch per stage over all slots of a batch; each slot uses up to 2 column
// blocks (32 right-hand sides), its own tile plan and its own buffers, so its
// result does not depend on the other slots.

__global__ __launch_bounds__(256) void colmax_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0 || S.prec != GPL_PREC_F16X3) return;
  const int local = blockIdx.x - B.off[s];
  colmax_body(local % kColmaxBlocks, local / kColmaxBlocks, S.N, S.T1, S.ldf, S.colmax);
}

__global__ void prep_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0) return;
  const int local = blockIdx.x - B.off[s];
  const int per = cdiv(S.ldh, 256);
  if (S.prec == GPL_PREC_F16X3)
    split_rhs_body(local % per, local / per, S.N, S.nrhs, S.T1, S.ldf, S.plan.perm, S.colmax, S.Vh, S.Vl, S.ldh,
                   S.inv_scale);
  else
    pack_rhs_body(local % per, local / per, S.N, S.nrhs, S.T1, S.ldf, S.plan.perm, S.Vp, S.ldh);
}

__global__ __launch_bounds__(256) void mvm_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0) return;
  const int item = blockIdx.x - B.off[s];
  if (S.prec == GPL_PREC_F16X3) {
    if (S.nrhs > 16)
      mvm_f16x3_item<2>(item, S.plan, S.s2, S.Vh, S.Vl, S.ldh, S.nrhs, S.part, S.nrhs, 0);
    else
      mvm_f16x3_item<1>(item, S.plan, S.s2, S.Vh, S.Vl, S.ldh, S.nrhs, S.part, S.nrhs, 0);
  } else {
    if (S.nrhs > 16)
      mvm_f32_item<2>(item, S.plan, S.s2, S.Vp, S.ldh, S.nrhs, S.part, S.nrhs, 0);
    else
      mvm_f32_item<1>(item, S.plan, S.s2, S.Vp, S.ldh, S.nrhs, S.part, S.nrhs, 0);
  }
}

__global__ void reduce_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0) return;
  const int local = blockIdx.x - B.off[s];
  const int per = cdiv(S.N, 256);
  reduce_body(local % per, local / per, S.plan, S.nrhs, S.part, S.nrhs,
              S.prec == GPL_PREC_F16X3 ? S.inv_scale : nullptr, S.amp2, S.T2, S.ldf, 0.f);
}

static int launch_grouped(void (*kern)(SlotBatch, int), const ServeSlotDev* const* hslots,
                          const ServeSlotDev* const* dslots, int nslots, int p, int (*blocks)(const ServeSlotDev&),
                          hipStream_t stream) {
  SlotBatch B;
  B.nslots = nslots;
  B.off[0] = 0;
  for (int s = 0; s < nslots; ++s) {
    B.slot[s] = dslots[s];
    B.off[s + 1] = B.off[s] + blocks(*hslots[s]);
  }
  if (B.off[nslots] == 0) return GPL_OK;
  hipLaunchKernelGGL(kern, dim3(B.off[nslots]), dim3(256), 0, stream, B, p);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int mvm_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                hipStream_t stream) {
  GPL_TRY(launch_grouped(colmax_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return S.prec == GPL_PREC_F16X3 ? kColmaxBlocks * S.nrhs : 0; },
                         stream));
  GPL_TRY(launch_grouped(prep_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return cdiv(S.ldh, 256) * S.ncp; }, stream));
  hipEvent_t t0 = timing_begin(stream);
  GPL_TRY(launch_grouped(mvm_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return S.plan.nrt * kMaxSeg; }, stream));
  timing_end(t0, stream);
  GPL_TRY(launch_grouped(reduce_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return cdiv(S.N, 256) * S.nrhs; }, stream));
  return GPL_OK;
}

}  // namespace gpl
