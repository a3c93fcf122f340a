// Kernel-matrix product on MFMA: Y = K V + beta Y with K_ij = a^2 exp(-|p_i-p_j|^2/(2 l^2))
// (eq. "grbf"), the exp tile formed in registers and contracted with the
// right-hand-side block on the matrix cores (the tile x RHS product is a true
// dense contraction).
//
// Work decomposition (both forms): a workgroup of 4 waves owns 256 output rows
// (each wave 4 row tiles of 16) and one slice of the source points. Source
// points and the RHS tile of 256 points are staged in LDS; every wave computes
// its exp values directly in the MFMA A-operand layout (lane = row within the
// tile; the lane's K slots = a run of consecutive source points, a permutation
// of K that the B operand shares), so no tile is ever written to memory. Exact
// coordinate differences are formed before scaling. Partial products of the
// slices are reduced in a fixed order by a second kernel (bitwise reproducible).
//
// Precision form (GPL_PREC_F16X3): exp tiles computed in FP32 as 2^11 k (the
// factor enters through the exp2 argument), split into FP16 hi (round toward
// zero) and lo = k - hi; the RHS block is pre-split the same way after a
// per-column power-of-two scale that puts its largest entry near 2^14. Each
// 16x16x32 tile takes three MFMAs (hi.hi + hi.lo + lo.hi) into FP32
// accumulators; the dropped lo.lo term is ~2^-22 relative.
//
// FP32 form on MFMA (GPL_PREC_FP32, several columns): the exp tile and the RHS
// in FP32 on v_mfma_f32_16x16x4_f32.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "common.hpp"
#include "internal.hpp"
#include "mvm_mfma.hpp"
#include "timing.hpp"

namespace gpl {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kJT = 256;                       // source points per LDS stage
constexpr int kRT = 4;                         // 16-row tiles per wave
constexpr int kWaves = 4;                      // waves per workgroup
constexpr int kRowsWG = kWaves * kRT * 16;     // rows per workgroup
constexpr float kKScale = 2048.f;              // 2^11 applied to the FP16 exp tile

struct MfmaPlan {
  int nrb, S, jlen, ldp, ldh, cb;
};

static MfmaPlan mfma_plan(int n, int nrhs) {
  MfmaPlan p;
  p.cb = cdiv(nrhs, 16);
  p.nrb = cdiv(n, kRowsWG);
  const int target = 2048;
  const int S = std::max(1, std::min(target / p.nrb, cdiv(n, kJT)));
  p.jlen = round_up(cdiv(n, S), kJT);
  p.S = cdiv(n, p.jlen);
  p.ldp = round_up(n, 64);
  p.ldh = round_up(n, kJT);
  return p;
}

// ---------------------------------------------------------------- RHS preparation

// Column-wise max |V| in two steps without atomics: kColmaxBlocks workgroups per
// column write partial maxima (as bit patterns of non-negative floats); the
// split kernel folds them (kColmaxBlocks workgroups per column).

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

// V' = V * 2^e_c split into FP16 hi (nearest) and lo; zero padding for j >= n
// and c >= nrhs; inv_scale[c] = 2^-e_c / 2^11 folds both scales for the output.
__device__ __forceinline__ void split_rhs_body(int bx, int c, int n, int nrhs, const float* __restrict__ V, int ldv,
                                               const unsigned* colmax, _Float16* Vh, _Float16* Vl, int ldh,
                                               float* inv_scale) {
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
  float v = (c < nrhs && j < n) ? V[(size_t)c * ldv + j] * scale : 0.f;
  const _Float16 h = (_Float16)v;
  const _Float16 l = (_Float16)(v - (float)h);
  Vh[(size_t)c * ldh + j] = h;
  Vl[(size_t)c * ldh + j] = l;
}

__global__ void split_rhs_kernel(int n, int nrhs, const float* __restrict__ V, int ldv, const unsigned* colmax,
                                 _Float16* Vh, _Float16* Vl, int ldh, float* inv_scale, CgGate gate) {
  if (gate.skip_all()) return;
  split_rhs_body(blockIdx.x, blockIdx.y, n, nrhs, V, ldv, colmax, Vh, Vl, ldh, inv_scale);
}

// ---------------------------------------------------------------- precision form

__device__ inline half8 pack_rtz(const float* k) {
  half8 r;
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const auto p = __builtin_amdgcn_cvt_pkrtz(k[e], k[e + 1]);
    half2v q = __builtin_bit_cast(half2v, p);
    r[e] = q[0];
    r[e + 1] = q[1];
  }
  return r;
}

template <int CB, int JT, bool RR>
__device__ __forceinline__ void mvm_f16x3_body(int bx, int by, int n, const float* __restrict__ px,
                                               const float* __restrict__ py, float s2,
                                               const _Float16* __restrict__ Vh, const _Float16* __restrict__ Vl,
                                               int ldh, int jlen, float* __restrict__ part, int ldp,
                                               int slice_cols) {
  constexpr int NCP = CB * 16;
  constexpr int LDSJ = JT + 8;  // halves per LDS row (padding against bank conflicts)
  __shared__ __attribute__((aligned(16))) float sxj[JT];
  __shared__ __attribute__((aligned(16))) float syj[JT];
  __shared__ __attribute__((aligned(16))) _Float16 sVh[NCP * LDSJ];
  __shared__ __attribute__((aligned(16))) _Float16 sVl[NCP * LDSJ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ri = lane & 15, g = lane >> 4;
  const int row_base = bx * kRowsWG + wave * (kRT * 16);
  float xi[kRT], yi[kRT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    const int i = row_base + rt * 16 + ri;
    xi[rt] = i < n ? px[i] : 0.f;
    yi[rt] = i < n ? py[i] : 0.f;
  }
  f32x4 acc[kRT][CB];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int jbeg = by * jlen;
  const int jend = min(n, jbeg + jlen);
  for (int jt = jbeg; jt < jend; jt += JT) {
    __syncthreads();
    for (int t = tid; t < JT; t += 256) {
      const int j = jt + t;
      sxj[t] = j < n ? px[j] : 0.f;
      syj[t] = j < n ? py[j] : 0.f;
    }
    // RHS tiles: NCP columns x JT points, 8 halves per load (buffers are padded
    // with zeros up to ldh >= jt + JT)
    for (int idx = tid; idx < NCP * (JT / 8); idx += 256) {
      const int c = idx / (JT / 8), j8 = (idx - c * (JT / 8)) * 8;
      *reinterpret_cast<half8*>(&sVh[c * LDSJ + j8]) =
          *reinterpret_cast<const half8*>(&Vh[(size_t)c * ldh + jt + j8]);
      *reinterpret_cast<half8*>(&sVl[c * LDSJ + j8]) =
          *reinterpret_cast<const half8*>(&Vl[(size_t)c * ldh + jt + j8]);
    }
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < JT / 32; ++s) {
      const int jl = s * 32 + g * 8;  // this lane's 8 consecutive source points
      float xj[8], yj[8];
      *reinterpret_cast<f32x4*>(&xj[0]) = *reinterpret_cast<const f32x4*>(&sxj[jl]);
      *reinterpret_cast<f32x4*>(&xj[4]) = *reinterpret_cast<const f32x4*>(&sxj[jl + 4]);
      *reinterpret_cast<f32x4*>(&yj[0]) = *reinterpret_cast<const f32x4*>(&syj[jl]);
      *reinterpret_cast<f32x4*>(&yj[4]) = *reinterpret_cast<const f32x4*>(&syj[jl + 4]);
      half8 bh[CB], bl[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int c = cb * 16 + ri;
        bh[cb] = *reinterpret_cast<const half8*>(&sVh[c * LDSJ + jl]);
        bl[cb] = *reinterpret_cast<const half8*>(&sVl[c * LDSJ + jl]);
      }
      if constexpr (RR) {
        // all row tiles' A operands first, then MFMAs round-robin over the
        // independent accumulators
        half8 ah[kRT], al[kRT];
#pragma unroll
        for (int rt = 0; rt < kRT; ++rt) {
          float k[8], lo[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float dx = xi[rt] - xj[e], dy = yi[rt] - yj[e];
            const float d2 = fmaf(dx, dx, dy * dy);
            k[e] = exp2_fast(fmaf(d2, -s2, 11.f));  // 2^11 k
          }
          ah[rt] = pack_rtz(k);
#pragma unroll
          for (int e = 0; e < 8; ++e) lo[e] = k[e] - (float)ah[rt][e];
          al[rt] = pack_rtz(lo);
        }
#pragma unroll
        for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[rt], bh[cb], acc[rt][cb], 0, 0, 0);
#pragma unroll
        for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[rt], bl[cb], acc[rt][cb], 0, 0, 0);
#pragma unroll
        for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[rt], bh[cb], acc[rt][cb], 0, 0, 0);
      } else {
#pragma unroll
        for (int rt = 0; rt < kRT; ++rt) {
          float k[8], lo[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float dx = xi[rt] - xj[e], dy = yi[rt] - yj[e];
            const float d2 = fmaf(dx, dx, dy * dy);
            k[e] = exp2_fast(fmaf(d2, -s2, 11.f));  // 2^11 k
          }
          const half8 hi = pack_rtz(k);
#pragma unroll
          for (int e = 0; e < 8; ++e) lo[e] = k[e] - (float)hi[e];
          const half8 lo8 = pack_rtz(lo);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, bh[cb], acc[rt][cb], 0, 0, 0);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, bl[cb], acc[rt][cb], 0, 0, 0);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo8, bh[cb], acc[rt][cb], 0, 0, 0);
        }
      }
    }
  }
  // D layout: column = lane % 16, rows 4 * (lane / 16) + v
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row_base + rt * 16 + g * 4 + v;
        const int c = cb * 16 + ri;
        if (i < n) part[((size_t)by * slice_cols + c) * ldp + i] = acc[rt][cb][v];
      }
}

template <int CB, int JT, bool RR>
__global__ __launch_bounds__(256) void mvm_f16x3_kernel(int n, const float* __restrict__ px,
                                                        const float* __restrict__ py, float s2,
                                                        const _Float16* __restrict__ Vh,
                                                        const _Float16* __restrict__ Vl, int ldh, int jlen,
                                                        float* __restrict__ part, int ldp, int slice_cols,
                                                        CgGate gate) {
  if (gate.skip_all()) return;
  mvm_f16x3_body<CB, JT, RR>(blockIdx.x, blockIdx.y, n, px, py, s2, Vh, Vl, ldh, jlen, part, ldp, slice_cols);
}

// ---------------------------------------------------------------- FP32 form on MFMA

template <int CB>
__device__ __forceinline__ void mvm_f32mfma_body(int bx, int by, int n, const float* __restrict__ px,
                                                 const float* __restrict__ py, float s2, const float* __restrict__ V,
                                                 int ldv, int nrhs, int jlen, float* __restrict__ part, int ldp,
                                                 int slice_cols) {
  constexpr int NCP = CB * 16;
  constexpr int LDSJ = kJT + 4;
  __shared__ __attribute__((aligned(16))) float sxj[kJT];
  __shared__ __attribute__((aligned(16))) float syj[kJT];
  __shared__ __attribute__((aligned(16))) float sV[NCP * LDSJ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ri = lane & 15, g = lane >> 4;
  const int row_base = bx * kRowsWG + wave * (kRT * 16);
  float xi[kRT], yi[kRT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    const int i = row_base + rt * 16 + ri;
    xi[rt] = i < n ? px[i] : 0.f;
    yi[rt] = i < n ? py[i] : 0.f;
  }
  f32x4 acc[kRT][CB];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int jbeg = by * jlen;
  const int jend = min(n, jbeg + jlen);
  for (int jt = jbeg; jt < jend; jt += kJT) {
    __syncthreads();
    {
      const int j = jt + tid;
      sxj[tid] = j < n ? px[j] : 0.f;
      syj[tid] = j < n ? py[j] : 0.f;
      const bool jok = j < jend;
      const float* vp = V + j;
#pragma unroll 1
      for (int c = 0; c < NCP; ++c, vp += ldv) sV[c * LDSJ + tid] = (c < nrhs && jok) ? *vp : 0.f;
    }
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < kJT / 16; ++s) {
      const int jl = s * 16 + g * 4;  // this lane's 4 consecutive source points
      const f32x4 xj = *reinterpret_cast<const f32x4*>(&sxj[jl]);
      const f32x4 yj = *reinterpret_cast<const f32x4*>(&syj[jl]);
      f32x4 b[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) b[cb] = *reinterpret_cast<const f32x4*>(&sV[(cb * 16 + ri) * LDSJ + jl]);
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt) {
        float k[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float dx = xi[rt] - xj[e], dy = yi[rt] - yj[e];
          const float d2 = fmaf(dx, dx, dy * dy);
          k[e] = exp2_fast(-(d2 * s2));
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(k[e], b[cb][e], acc[rt][cb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row_base + rt * 16 + g * 4 + v;
        const int c = cb * 16 + ri;
        if (i < n) part[((size_t)by * slice_cols + c) * ldp + i] = acc[rt][cb][v];
      }
}

template <int CB>
__global__ __launch_bounds__(256) void mvm_f32mfma_kernel(int n, const float* __restrict__ px,
                                                          const float* __restrict__ py, float s2,
                                                          const float* __restrict__ V, int ldv, int nrhs, int jlen,
                                                          float* __restrict__ part, int ldp, int slice_cols,
                                                          CgGate gate) {
  if (gate.skip_all()) return;
  mvm_f32mfma_body<CB>(blockIdx.x, blockIdx.y, n, px, py, s2, V, ldv, nrhs, jlen, part, ldp, slice_cols);
}

// Y[c] = (amp2 * colscale[c]) * sum_s part[s][c] + beta Y[c], slices in order.
__device__ __forceinline__ void mfma_reduce_body(int bx, int c, int n, int nrhs, int ncp, int S,
                                                 const float* __restrict__ part, int ldp,
                                                 const float* __restrict__ colscale, float amp2, float* Y, int ldy,
                                                 float beta) {
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= n || c >= nrhs) return;
  float s = 0.f;
  for (int k = 0; k < S; ++k) s += part[((size_t)k * ncp + c) * ldp + i];
  const float f = colscale ? amp2 * colscale[c] : amp2;
  float* y = Y + (size_t)c * ldy + i;
  const float res = f * s;
  *y = beta != 0.f ? res + beta * *y : res;
}

__global__ void mfma_reduce_kernel(int n, int nrhs, int ncp, int S, const float* __restrict__ part, int ldp,
                                   const float* __restrict__ colscale, float amp2, float* Y, int ldy, float beta,
                                   CgGate gate) {
  if (gate.skip_all()) return;
  mfma_reduce_body(blockIdx.x, blockIdx.y, n, nrhs, ncp, S, part, ldp, colscale, amp2, Y, ldy, beta);
}

// ---------------------------------------------------------------- grouped launches (serving)
// One launch per stage over all slots of a batch; each slot uses 2 column
// blocks (up to 32 right-hand sides) and its own slice plan, so its result does
// not depend on the other slots.

__global__ __launch_bounds__(256) void colmax_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0 || S.prec != GPL_PREC_F16X3) return;
  const int local = blockIdx.x - B.off[s];
  colmax_body(local % kColmaxBlocks, local / kColmaxBlocks, S.N, S.T1, S.ldf, S.colmax);
}

__global__ void split_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0 || S.prec != GPL_PREC_F16X3) return;
  const int local = blockIdx.x - B.off[s];
  const int per = (S.ldh + 255) / 256;
  split_rhs_body(local % per, local / per, S.N, S.nrhs, S.T1, S.ldf, S.colmax, S.Vh, S.Vl, S.ldh, S.inv_scale);
}

__global__ __launch_bounds__(256) void mvm_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0) return;
  const int local = blockIdx.x - B.off[s];
  const int bx = local % S.nrb, by = local / S.nrb;
  if (S.prec == GPL_PREC_F16X3)
    mvm_f16x3_body<2, 256, false>(bx, by, S.N, S.px, S.py, S.s2, S.Vh, S.Vl, S.ldh, S.jlen, S.part, S.ldp, 32);
  else
    mvm_f32mfma_body<2>(bx, by, S.N, S.px, S.py, S.s2, S.T1, S.ldf, S.nrhs, S.jlen, S.part, S.ldp, 32);
}

__global__ void reduce_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0) return;
  const int local = blockIdx.x - B.off[s];
  const int per = (S.N + 255) / 256;
  mfma_reduce_body(local % per, local / per, S.N, S.nrhs, 32, S.S, S.part, S.ldp,
                   S.prec == GPL_PREC_F16X3 ? S.inv_scale : nullptr, S.amp2, S.T2, S.ldf, 0.f);
}

// ---------------------------------------------------------------- host side

template <class C>
static void carve_f16x3(C& cv, const MfmaPlan& p, unsigned** colmax, float** inv_scale, _Float16** Vh, _Float16** Vl,
                        float** part) {
  const int ncp = p.cb * 16;
  *colmax = cv.template take<unsigned>((size_t)ncp * kColmaxBlocks);
  *inv_scale = cv.template take<float>(ncp);
  *Vh = cv.template take<_Float16>((size_t)ncp * p.ldh);
  *Vl = cv.template take<_Float16>((size_t)ncp * p.ldh);
  *part = cv.template take<float>((size_t)p.S * ncp * p.ldp);
}

size_t mfma_f16x3_workspace(int n, int nrhs) {
  if (n <= 0 || nrhs <= 0) return 0;
  const MfmaPlan p = mfma_plan(n, nrhs);
  Sizer s;
  unsigned* a;
  float *b, *e;
  _Float16 *c, *d;
  carve_f16x3(s, p, &a, &b, &c, &d, &e);
  return s.used;
}

template <int CB, int JT, bool RR>
static void launch_f16x3_v(const MfmaPlan& p, int n, const float* px, const float* py, float s2, const _Float16* Vh,
                           const _Float16* Vl, float* part, CgGate gate, hipStream_t stream) {
  hipLaunchKernelGGL((mvm_f16x3_kernel<CB, JT, RR>), dim3(p.nrb, p.S), dim3(256), 0, stream, n, px, py, s2, Vh, Vl,
                     p.ldh, p.jlen, part, p.ldp, p.cb * 16, gate);
}

template <int CB>
static void launch_f16x3(const MfmaPlan& p, int n, const float* px, const float* py, float s2, const _Float16* Vh,
                         const _Float16* Vl, float* part, CgGate gate, hipStream_t stream) {
  static const int env_v = getenv("GPLENS_F16X3_VARIANT") ? atoi(getenv("GPLENS_F16X3_VARIANT")) : -1;
  const int v = env_v >= 0 ? env_v : (CB >= 3 ? 2 : 0);
  switch (v & 3) {
    case 0: launch_f16x3_v<CB, 256, false>(p, n, px, py, s2, Vh, Vl, part, gate, stream); break;
    case 1: launch_f16x3_v<CB, 256, true>(p, n, px, py, s2, Vh, Vl, part, gate, stream); break;
    case 2: launch_f16x3_v<CB, 128, false>(p, n, px, py, s2, Vh, Vl, part, gate, stream); break;
    default: launch_f16x3_v<CB, 128, true>(p, n, px, py, s2, Vh, Vl, part, gate, stream); break;
  }
}

static constexpr int kMaxCB = 4;  // up to 64 columns per pass

int mfma_f16x3_launch(float s2, float amp2, int n, const float* px, const float* py, int nrhs, const float* V, int ldv,
                      float* Y, int ldy, float beta, void* ws, size_t ws_bytes, CgGate gate, hipStream_t stream) {
  GPL_TRY(check_ws(ws, ws_bytes, mfma_f16x3_workspace(n, nrhs)));
  const MfmaPlan p = mfma_plan(n, nrhs);
  Carver cv(ws, ws_bytes);
  unsigned* colmax;
  float *inv_scale, *part;
  _Float16 *Vh, *Vl;
  carve_f16x3(cv, p, &colmax, &inv_scale, &Vh, &Vl, &part);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  const int ncp = p.cb * 16;
  hipLaunchKernelGGL(colmax_kernel, dim3(kColmaxBlocks, nrhs), dim3(256), 0, stream, n, V, ldv, colmax, gate);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(split_rhs_kernel, dim3(cdiv(p.ldh, 256), ncp), dim3(256), 0, stream, n, nrhs, V, ldv, colmax, Vh,
                     Vl, p.ldh, inv_scale, gate);
  GPL_LAUNCH_CHECK();
  // column blocks of up to 64 columns per pass; each pass writes its own part rows
  for (int c0 = 0; c0 < ncp; c0 += kMaxCB * 16) {
    const int cb = std::min(kMaxCB, (ncp - c0) / 16);
    const _Float16* vh = Vh + (size_t)c0 * p.ldh;
    const _Float16* vl = Vl + (size_t)c0 * p.ldh;
    // part layout [S][ncp][ldp]; this pass writes columns c0 .. c0 + 16 cb of every slice
    float* pp = part + (size_t)c0 * p.ldp;
    hipEvent_t t0 = timing_begin(stream);
    switch (cb) {
      case 4: launch_f16x3<4>(p, n, px, py, s2, vh, vl, pp, gate, stream); break;
      case 3: launch_f16x3<3>(p, n, px, py, s2, vh, vl, pp, gate, stream); break;
      case 2: launch_f16x3<2>(p, n, px, py, s2, vh, vl, pp, gate, stream); break;
      default: launch_f16x3<1>(p, n, px, py, s2, vh, vl, pp, gate, stream); break;
    }
    GPL_LAUNCH_CHECK();
    timing_end(t0, stream);
  }
  hipLaunchKernelGGL(mfma_reduce_kernel, dim3(cdiv(n, 256), nrhs), dim3(256), 0, stream, n, nrhs, ncp, p.S, part,
                     p.ldp, inv_scale, amp2, Y, ldy, beta, gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

void serve_mvm_plan(int N, int* S, int* jlen, int* nrb, int* ldh, int* ldp) {
  const MfmaPlan p = mfma_plan(N, 32);
  *S = p.S;
  *jlen = p.jlen;
  *nrb = p.nrb;
  *ldh = p.ldh;
  *ldp = p.ldp;
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
  GPL_TRY(launch_grouped(split_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return S.prec == GPL_PREC_F16X3 ? (S.ldh + 255) / 256 * 32 : 0; },
                         stream));
  hipEvent_t t0 = timing_begin(stream);
  GPL_TRY(launch_grouped(mvm_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return S.nrb * S.S; }, stream));
  timing_end(t0, stream);
  GPL_TRY(launch_grouped(reduce_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return (S.N + 255) / 256 * S.nrhs; }, stream));
  return GPL_OK;
}

size_t mfma_f32_workspace(int n, int nrhs) {
  if (n <= 0 || nrhs <= 0) return 0;
  const MfmaPlan p = mfma_plan(n, nrhs);
  return align_up(sizeof(float) * (size_t)p.S * p.cb * 16 * p.ldp);
}

template <int CB>
static void launch_f32mfma(const MfmaPlan& p, int n, const float* px, const float* py, float s2, const float* V,
                           int ldv, int ncols, float* part, CgGate gate, hipStream_t stream) {
  hipLaunchKernelGGL((mvm_f32mfma_kernel<CB>), dim3(p.nrb, p.S), dim3(256), 0, stream, n, px, py, s2, V, ldv, ncols,
                     p.jlen, part, p.ldp, p.cb * 16, gate);
}

int mfma_f32_launch(float s2, float amp2, int n, const float* px, const float* py, int nrhs, const float* V, int ldv,
                    float* Y, int ldy, float beta, void* ws, size_t ws_bytes, CgGate gate, hipStream_t stream) {
  GPL_TRY(check_ws(ws, ws_bytes, mfma_f32_workspace(n, nrhs)));
  const MfmaPlan p = mfma_plan(n, nrhs);
  float* part = static_cast<float*>(ws);
  const int ncp = p.cb * 16;
  for (int c0 = 0; c0 < ncp; c0 += kMaxCB * 16) {
    const int cb = std::min(kMaxCB, (ncp - c0) / 16);
    const float* v = V + (size_t)c0 * ldv;
    float* pp = part + (size_t)c0 * p.ldp;
    const int ncols = std::min(nrhs - c0, cb * 16);
    hipEvent_t t0 = timing_begin(stream);
    switch (cb) {
      case 4: launch_f32mfma<4>(p, n, px, py, s2, v, ldv, ncols, pp, gate, stream); break;
      case 3: launch_f32mfma<3>(p, n, px, py, s2, v, ldv, ncols, pp, gate, stream); break;
      case 2: launch_f32mfma<2>(p, n, px, py, s2, v, ldv, ncols, pp, gate, stream); break;
      default: launch_f32mfma<1>(p, n, px, py, s2, v, ldv, ncols, pp, gate, stream); break;
    }
    GPL_LAUNCH_CHECK();
    timing_end(t0, stream);
  }
  hipLaunchKernelGGL(mfma_reduce_kernel, dim3(cdiv(n, 256), nrhs), dim3(256), 0, stream, n, nrhs, ncp, p.S, part,
                     p.ldp, nullptr, amp2, Y, ldy, beta, gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl
