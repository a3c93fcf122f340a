// Kernel-matrix product on MFMA: Y = K V + beta Y with K_ij = a^2 exp(-|p_i-p_j|^2/(2 l^2))
// (eq. "grbf"), the exp tile formed in registers and contracted with the
// right-hand-side block on the matrix cores (the tile x RHS product is a true
// dense contraction). K is never stored (Sec. 3.3).
//
// Work decomposition: the points are taken in the order of a tile plan
// (tileplan.hpp), which lists for every row tile of 64 points the chunks of 32
// points that can give a non-zero kernel value, each with the mask of the row
// tile's four 16-point subtiles that can; every other pair contributes exact
// zeros and is not evaluated (a masked-out subtile skips its exp tile and
// MFMAs). The listed (row tile, chunk) pairs are split over the waves of the
// launch by an estimate of their cost, each wave taking a contiguous run of them
// (so the work is balanced however unevenly the live pairs fall on row tiles).
// A wave computes 64 rows (four 16-row MFMA tiles) at a time, with each chunk's
// coordinates and right-hand-side block loaded straight from global memory into
// the MFMA B-operand layout, and writes one block of partial rows per row tile
// it touches; a reduction kernel adds the partials of each row tile in wave
// order and scatters to the caller's order, so the result is bitwise
// reproducible. Exact coordinate differences are formed before scaling.
//
// Precision form (GPL_PREC_F16X3): exp tiles computed in FP32 as 2^11 k (the
// factor enters through the exp2 argument) and split into FP16 hi (truncated
// toward zero) and lo = k - hi (exact in FP32); the RHS block is split after
// a per-column power-of-two scale that puts its largest entry near 2^14. Each
// 16x16x32 tile takes three MFMAs (hi.hi + hi.lo + lo.hi) into FP32
// accumulators; the dropped lo.lo term is ~2^-22 relative. A last block of at
// most 8 columns is packed (hi and lo of a column side by side, see hi_slot)
// and takes two: hi.[hi lo] + lo.[hi lo].
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

constexpr int kRT = kSubsPerTile;           // 16-row MFMA tiles per wave
constexpr int kWaves = 4;                   // independent waves per workgroup
constexpr float kKScale = 2048.f;           // 2^11 applied to the FP16 exp tile
static constexpr int kMaxCB = 4;            // up to 64 columns per pass

static_assert(kRT * 16 == kRowTile, "row tile of 16-row MFMA tiles");

static_assert(kWaves == kPlanWaves, "the plan orders workgroups of kPlanWaves waves");

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
__device__ __forceinline__ void split_rhs_body(int bx, int slot, int n, int nrhs, const float* __restrict__ V,
                                               int ldv, const int* perm, const unsigned* colmax, _Float16* Vh,
                                               _Float16* Vl, int ldh, int ncp, float* inv_scale) {
  const int j = bx * blockDim.x + threadIdx.x;
  if (j >= ldh) return;
  // slot `slot` of the buffers: column `slot`, or in a packed last block one
  // FP16 part (lo in odd slots) of column b0 + (slot - b0) / 2
  const int b0 = packed_block_start(nrhs);
  const bool packed = last_block_packed(nrhs) && slot >= b0;
  const int c = packed ? b0 + (slot - b0) / 2 : slot;
  int e = 0;
  if (c < nrhs) {
    unsigned mb = 0u;
    for (int b = 0; b < kColmaxBlocks; ++b) mb = max(mb, colmax[c * kColmaxBlocks + b]);
    const float mx = __uint_as_float(mb);
    // mx * 2^e in [2^13, 2^14); e is capped so that 2^e stays a finite float
    // (a column below 2^-113 then scales to less than 2^13, still normal in FP16)
    if (mx > 0.f && isfinite(mx)) e = min(14 - ilogbf(mx) - 1, 126);
  }
  const float scale = ldexpf(1.f, e);
  if (j == 0 && c < ncp && (!packed || ((slot - b0) & 1) == 0)) inv_scale[c] = ldexpf(1.f, -e) / kKScale;
  const float v = gather_rhs(j, c, n, nrhs, perm, V, ldv) * scale;
  const _Float16 h = (_Float16)v;
  const _Float16 l = (_Float16)(v - (float)h);
  if (packed) {
    Vh[rhs_at(slot, j, ncp)] = ((slot - b0) & 1) ? l : h;
  } else {
    Vh[rhs_at(c, j, ncp)] = h;
    Vl[rhs_at(c, j, ncp)] = l;
  }
}

__global__ void split_rhs_kernel(int n, int nrhs, const float* __restrict__ V, int ldv, const int* perm,
                                 const unsigned* colmax, _Float16* Vh, _Float16* Vl, int ldh, int ncp, float* inv_scale,
                                 CgGate gate) {
  if (gate.skip_all()) return;
  split_rhs_body(blockIdx.x, blockIdx.y, n, nrhs, V, ldv, perm, colmax, Vh, Vl, ldh, ncp, inv_scale);
}

// FP32 form: the RHS block in sorted order, zero padded.
__device__ __forceinline__ void pack_rhs_body(int bx, int c, int n, int nrhs, const float* __restrict__ V, int ldv,
                                              const int* perm, float* Vp, int ldh, int ncp) {
  const int j = bx * blockDim.x + threadIdx.x;
  if (j >= ldh) return;
  Vp[rhs_at(c, j, ncp)] = gather_rhs(j, c, n, nrhs, perm, V, ldv);
}

__global__ void pack_rhs_kernel(int n, int nrhs, const float* __restrict__ V, int ldv, const int* perm, float* Vp,
                                int ldh, int ncp, CgGate gate) {
  if (gate.skip_all()) return;
  pack_rhs_body(blockIdx.x, blockIdx.y, n, nrhs, V, ldv, perm, Vp, ldh, ncp);
}

// ---------------------------------------------------------------- work of one wave

// Partial rows of one row tile from one wave: part[(slot * pcols + c0 + c) * 64 + row]
// for c < ncols (MFMA D layout: column = lane % 16, rows 4 * (lane / 16) + v). In a
// packed last block (PK) accumulator columns 2t and 2t + 1 (lanes ri, ri + 1) are
// the two parts of column 16 (CB - 1) + t and are added.
template <int CB, bool PK>
__device__ __forceinline__ void store_partial(const f32x4 (&acc)[kRT][CB], int slot, float* __restrict__ part,
                                              int pcols, int c0, int ncols, int ri, int g) {
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      f32x4 v = acc[rt][cb];
      int c = cb * 16 + ri;
      if (PK && cb == CB - 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += __shfl_down(v[k], 1, 64);
        c = (ri & 1) ? ncols : cb * 16 + ri / 2;  // odd lanes hold the second parts
      }
      if (c < ncols)
        *reinterpret_cast<f32x4*>(&part[((size_t)slot * pcols + c0 + c) * kRowTile + rt * 16 + g * 4]) = v;
    }
}

// Runs `body(entry)` for the list entries at positions [kb, ke) of a row tile's
// list; the entries are read 64 at a time, one per lane, and broadcast with
// readlane so that the chunk and its subtile mask are uniform across the wave.
template <class F>
__device__ __forceinline__ void for_chunks(const uint32_t* lst, int kb, int ke, int lane, F&& body) {
#pragma unroll 1
  for (int k0 = kb; k0 < ke; k0 += 64) {
    const int m = min(64, ke - k0);
    const int vidx = lane < m ? (int)lst[k0 + lane] : 0;
#pragma unroll 1
    for (int t = 0; t < m; ++t) body((uint32_t)__builtin_amdgcn_readlane(vidx, t));
  }
}

// Waits until at most N vector-memory loads of this wave are outstanding (vmcnt
// only; the expcnt and lgkmcnt fields are left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// As for_chunks with two operand buffers: the next chunk's loads are issued
// before the current chunk is computed (a load past the end repeats the last
// chunk and is not used). Before each compute the wave waits explicitly for the
// current buffer, leaving exactly the next buffer's Buf::kLoads loads in flight;
// without it, the compiler's conservative waits at the subtile branches also
// waited for the next buffer and serialised every chunk on its loads.
template <class Buf, class L, class C>
__device__ __forceinline__ void for_chunks_pf(const uint32_t* lst, int kb, int ke, int lane, L&& load, C&& compute) {
#pragma unroll 1
  for (int k0 = kb; k0 < ke; k0 += 64) {
    const int m = min(64, ke - k0);
    const int vidx = lane < m ? (int)lst[k0 + lane] : 0;
    Buf a, b;
    load(a, (uint32_t)__builtin_amdgcn_readlane(vidx, 0));
#pragma unroll 1
    for (int t = 0; t < m; t += 2) {
      load(b, (uint32_t)__builtin_amdgcn_readlane(vidx, min(t + 1, m - 1)));
      __builtin_amdgcn_sched_barrier(0);  // keep the next chunk's loads ahead of this compute
      wait_vmcnt<Buf::kLoads>();
      compute(a);
      if (t + 1 >= m) break;
      load(a, (uint32_t)__builtin_amdgcn_readlane(vidx, min(t + 2, m - 1)));
      __builtin_amdgcn_sched_barrier(0);
      wait_vmcnt<Buf::kLoads>();
      compute(b);
    }
  }
}

// One wave's share of a product: for each row tile its units touch, load the
// tile's 64 row coordinates (from rx, ry), accumulate over the tile's chunks in
// the range, and write the partial rows. `chunk_fn(acc, xi, yi, r, lst, kb, ke,
// lane)` accumulates list positions [kb, ke) of row tile r. The wave's range comes from one
// descriptor load, issued together with the gate flag; `skip()` is evaluated
// once both are in.
template <int CB, bool PK, class S, class F>
__device__ __forceinline__ void wave_product(int w, const TilePlan& P, const float* __restrict__ rx,
                                             const float* __restrict__ ry, float* __restrict__ part, int pcols, int c0,
                                             int ncols, S&& skip, F&& chunk_fn) {
  const int4 d = P.wdesc[w];
  int rest = P.wrest[w];
  if (skip() || d.x < 0) return;
  const int lane = threadIdx.x & 63, ri = lane & 15, g = lane >> 4;
  int r = d.x, slot = d.y, kb = d.z, ke = d.w;
#pragma unroll 1
  while (true) {
    float xi[kRT], yi[kRT];
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      const int i = r * kRowTile + rt * 16 + ri;
      xi[rt] = rx[i];
      yi[rt] = ry[i];
    }
    f32x4 acc[kRT][CB];
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    chunk_fn(acc, xi, yi, r, P.list + (size_t)r * P.nch, kb, ke, lane);
    store_partial<CB, PK>(acc, slot, part, pcols, c0, ncols, ri, g);
    if (rest <= 0) break;
    ++r;
    ++slot;
    kb = 0;
    ke = min(rest, P.count[r]);
    rest -= ke;
  }
}

// ---------------------------------------------------------------- precision form

// Operands of one chunk for one lane: its 8 consecutive source points (scaled
// and block-centred), the hi/lo RHS fragments of every column block (columns
// past nrhs are zero), and the (uniform) centre of the chunk's block and mask of
// the subtiles that see the chunk.
template <int CB, bool PK>
struct F16Chunk {
  static constexpr int kLo = CB - (PK ? 1 : 0);  // blocks with a separate lo fragment
  static constexpr int kLoads = 5 + CB + kLo;    // vector loads issued by f16_load
  f32x4 x0, x1, y0, y1;
  half8 bh[CB], bl[kLo > 0 ? kLo : 1];
  float2 cen;
  unsigned mask, lomask;
};

// With FILT, a chunk whose generation differs from gen (its right-hand side is
// zero in every column) gets an empty subtile mask, so its tiles are not
// evaluated, and its loads read chunk 0 instead (they are still issued, which
// keeps the wait counts exact, but hit in cache).
template <int CB, bool PK, bool FILT = false>
__device__ __forceinline__ void f16_load(F16Chunk<CB, PK>& c, const TilePlan& P, const _Float16* __restrict__ Vh,
                                         const _Float16* __restrict__ Vl, int ncp, uint32_t entry, int ri, int g,
                                         const int* __restrict__ cgen = nullptr, int gen = 0) {
  c.mask = entry_mask(entry);
  if (FILT && cgen[entry_chunk(entry)] != gen) {
    c.mask = 0u;
    entry = 0u;
  }
  c.lomask = entry_lomask(entry);
  c.cen = P.cen[entry_chunk(entry) / kChunksPerTile];  // uniform address, one vector load
  const int j0 = entry_chunk(entry) * kChunk + g * 8;
  c.x0 = *reinterpret_cast<const f32x4*>(&P.xc[j0]);
  c.x1 = *reinterpret_cast<const f32x4*>(&P.xc[j0 + 4]);
  c.y0 = *reinterpret_cast<const f32x4*>(&P.yc[j0]);
  c.y1 = *reinterpret_cast<const f32x4*>(&P.yc[j0 + 4]);
  // uniform chunk base plus a fixed lane offset: little per-chunk address arithmetic
  const size_t cbase = (size_t)entry_chunk(entry) * ncp * kChunk;
  const _Float16* vh = Vh + cbase;
  const _Float16* vl = Vl + cbase;
  const unsigned lo = ri * kChunk + g * 8;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    c.bh[cb] = *reinterpret_cast<const half8*>(vh + cb * 16 * kChunk + lo);
    if (cb < F16Chunk<CB, PK>::kLo) c.bl[cb] = *reinterpret_cast<const half8*>(vl + cb * 16 * kChunk + lo);
  }
}

template <int CB, bool PK>
__device__ __forceinline__ void f16_compute(f32x4 (&acc)[kRT][CB], const F16Chunk<CB, PK>& c, const float (&xi)[kRT],
                                            const float (&yi)[kRT], float2 rcen) {
  // scaled differences: (xi + (centre_i - centre_j)) - xj, the centre
  // difference exact (both multiples of 2^-12) and uniform over the chunk
  const float ox = rcen.x - c.cen.x, oy = rcen.y - c.cen.y;
  const float xj[8] = {c.x0[0], c.x0[1], c.x0[2], c.x0[3], c.x1[0], c.x1[1], c.x1[2], c.x1[3]};
  const float yj[8] = {c.y0[0], c.y0[1], c.y0[2], c.y0[3], c.y1[0], c.y1[1], c.y1[2], c.y1[3]};
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    if (!((c.mask >> rt) & 1u)) continue;  // every exp of this 16 x 32 tile is exactly zero
    float lf[8], dx[8], dy[8], a[8], k2[8];
    const float xe = xi[rt] + ox, ye = yi[rt] + oy;
#pragma unroll
    for (int e = 0; e < 8; ++e) dx[e] = xe - xj[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) dy[e] = ye - yj[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = fmaf(-dy[e], dy[e], 11.f);
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = fmaf(-dx[e], dx[e], a[e]);  // 11 - s2 d^2
#pragma unroll
    for (int e = 0; e < 8; ++e) k2[e] = exp2_fast(a[e]);  // 2^11 k
    // hi = 2^11 k truncated to FP16
    half8 hi;
    decltype(__builtin_amdgcn_cvt_pkrtz(0.f, 0.f)) hp[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      hp[e / 2] = __builtin_amdgcn_cvt_pkrtz(k2[e], k2[e + 1]);
      const half2v h = __builtin_bit_cast(half2v, hp[e / 2]);
      hi[e] = h[0];
      hi[e + 1] = h[1];
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
      acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, c.bh[cb], acc[rt][cb], 0, 0, 0);
#pragma unroll
    for (int cb = 0; cb < F16Chunk<CB, PK>::kLo; ++cb)
      acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, c.bl[cb], acc[rt][cb], 0, 0, 0);
    if (!((c.lomask >> rt) & 1u)) continue;  // every k of the tile <= 2^-20: lo below 2^-30
    // lo = 2^11 k - hi exactly, formed from the FP16 half in one v_fma_mix_f32
    // (no compiler builtin selects it)
    half8 lo;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lf[e]) : "v"(hp[e / 2]), "v"(k2[e]));
      asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
          : "=v"(lf[e + 1])
          : "v"(hp[e / 2]), "v"(k2[e + 1]));
      const half2v l = __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(lf[e], lf[e + 1]));
      lo[e] = l[0];
      lo[e + 1] = l[1];
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
      acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo, c.bh[cb], acc[rt][cb], 0, 0, 0);
  }
}

template <int CB, bool PK, bool FILT = false, class Skip>
__device__ __forceinline__ void mvm_f16x3_wave(Skip&& skip, int w, const TilePlan& P, const _Float16* __restrict__ Vh,
                                               const _Float16* __restrict__ Vl, int ncp, int ncols,
                                               float* __restrict__ part, int pcols, int c0,
                                               const int* __restrict__ cgen = nullptr, int gen = 0) {
  const int lane = threadIdx.x & 63, ri = lane & 15, g = lane >> 4;
  wave_product<CB, PK>(w, P, P.xc, P.yc, part, pcols, c0, ncols, skip,
                   [&](f32x4 (&acc)[kRT][CB], const float (&xi)[kRT], const float (&yi)[kRT], int r,
                       const uint32_t* lst, int kb, int ke, int lane) {
                     const float2 rcen = P.cen[r];
                     for_chunks_pf<F16Chunk<CB, PK>>(lst, kb, ke, lane,
                         [&](F16Chunk<CB, PK>& c, uint32_t e) {
                           f16_load<CB, PK, FILT>(c, P, Vh, Vl, ncp, e, ri, g, cgen, gen);
                         },
                         [&](const F16Chunk<CB, PK>& c) { f16_compute(acc, c, xi, yi, rcen); });
                   });
}

// One wave per share of the plan's units; 4 independent waves per workgroup.
template <int CB, bool PK, bool FILT = false>
__global__ __launch_bounds__(256) void mvm_f16x3_kernel(const TilePlan P, const _Float16* __restrict__ Vh,
                                                        const _Float16* __restrict__ Vl, int ncp, int ncols,
                                                        float* __restrict__ part, int pcols, int c0, CgGate gate) {
  const int w = plan_block(blockIdx.x, P.nw, P.wround) * kWaves +
                __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  mvm_f16x3_wave<CB, PK, FILT>([&] { return gate.skip_all(); }, w, P, Vh, Vl, ncp, ncols, part, pcols, c0,
                               gate.chunk_gen, gate.gen);
}

// ---------------------------------------------------------------- FP32 form

template <int CB>
__device__ __forceinline__ void f32_chunk(f32x4 (&acc)[kRT][CB], const float (&xi)[kRT], const float (&yi)[kRT],
                                          const TilePlan& P, float s2, const float* __restrict__ Vp, int ncp,
                                          uint32_t entry, int ri, int g) {
  // two groups of 16 points; in each, this lane's 4 consecutive points
  const unsigned mask = entry_mask(entry);
  const int jc = entry_chunk(entry) * kChunk + g * 4;
  float xj[8], yj[8];
  *reinterpret_cast<f32x4*>(&xj[0]) = *reinterpret_cast<const f32x4*>(&P.xs[jc]);
  *reinterpret_cast<f32x4*>(&xj[4]) = *reinterpret_cast<const f32x4*>(&P.xs[jc + 16]);
  *reinterpret_cast<f32x4*>(&yj[0]) = *reinterpret_cast<const f32x4*>(&P.ys[jc]);
  *reinterpret_cast<f32x4*>(&yj[4]) = *reinterpret_cast<const f32x4*>(&P.ys[jc + 16]);
  const float* vp = Vp + (size_t)entry_chunk(entry) * ncp * kChunk;  // uniform chunk base
  const unsigned lo = ri * kChunk + g * 4;
  f32x4 b[CB][2];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int h = 0; h < 2; ++h) b[cb][h] = *reinterpret_cast<const f32x4*>(vp + cb * 16 * kChunk + 16 * h + lo);
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    if (!((mask >> rt) & 1u)) continue;  // every exp of this 16 x 32 tile is exactly zero
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

template <int CB, class Skip>
__device__ __forceinline__ void mvm_f32_wave(Skip&& skip, int w, const TilePlan& P, float s2, const float* __restrict__ Vp,
                                             int ncp, int ncols, float* __restrict__ part, int pcols, int c0) {
  const int lane = threadIdx.x & 63, ri = lane & 15, g = lane >> 4;
  wave_product<CB, false>(w, P, P.xs, P.ys, part, pcols, c0, ncols, skip,
                   [&](f32x4 (&acc)[kRT][CB], const float (&xi)[kRT], const float (&yi)[kRT], int,
                       const uint32_t* lst, int kb, int ke, int lane) {
                     for_chunks(lst, kb, ke, lane,
                                [&](uint32_t e) { f32_chunk<CB>(acc, xi, yi, P, s2, Vp, ncp, e, ri, g); });
                   });
}

template <int CB>
__global__ __launch_bounds__(256) void mvm_f32_kernel(const TilePlan P, float s2, const float* __restrict__ Vp,
                                                      int ncp, int ncols, float* __restrict__ part, int pcols, int c0,
                                                      CgGate gate) {
  const int w = plan_block(blockIdx.x, P.nw, P.wround) * kWaves +
                __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  mvm_f32_wave<CB>([&] { return gate.skip_all(); }, w, P, s2, Vp, ncp, ncols, part, pcols, c0);
}

// ---------------------------------------------------------------- reduction

// Y[c][perm[j]] = (amp2 * colscale[c]) * sum_q part[s0 + q][c][row] + beta Y over the
// partial slots [s0, s0 + cnt) of row tile r = j / 64, in wave order. A
// workgroup takes 256 points and KC columns, c0 = cg KC on; each wave's 64
// points are one row tile, so its slot range is uniform. KC = 4 halves the
// instructions per entry of a large product; a small one, bound by latency,
// runs faster with more waves (KC = 1).
// `skip()` is evaluated once the slot range and the destination index are loaded.
template <int KC, class Skip>
__device__ __forceinline__ void reduce_body(Skip&& skip, int bx, int cg, const TilePlan& P, int nrhs,
                                            const float* __restrict__ part, int pcols,
                                            const float* __restrict__ colscale, float amp2, float* Y, int ldy,
                                            float beta) {
  const int j0 = bx * 256 + (int)(threadIdx.x & ~63u);  // the wave's first point
  if (j0 >= P.n) return;
  const int r = j0 / kRowTile, row = threadIdx.x & 63, j = j0 + row;
  const int2 sl = P.rslot[r];
  const int dst = P.perm ? P.perm[min(j, P.n - 1)] : j;
  const int c0 = cg * KC;
  if (skip()) return;
  // the slot range is uniform over the wave; with one column a thread, the
  // per-lane values keep the addresses independent of a wave-wide wait
  const int s0 = KC > 1 ? __builtin_amdgcn_readfirstlane(sl.x) : sl.x;
  const int cnt = KC > 1 ? __builtin_amdgcn_readfirstlane(sl.y) : sl.y;
  const size_t stride = (size_t)pcols * kRowTile;
  const float* p0 = part + (size_t)s0 * stride + row;
  int coff[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) coff[k] = min(c0 + k, nrhs - 1) * kRowTile;
  // in slot order; the loads of each group of 8 slots are issued together. Past
  // the last slot (or column) a load repeats the last one (always a valid
  // address) and its value is not added: a load under a condition would be
  // branched around and waited for on its own.
  float acc[KC] = {};
  for (int q = 0; q < cnt; q += 8) {
    float t[8][KC];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float* ps = p0 + (size_t)min(q + u, cnt - 1) * stride;
#pragma unroll
      for (int k = 0; k < KC; ++k) t[u][k] = ps[coff[k]];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q + u < cnt)
#pragma unroll
        for (int k = 0; k < KC; ++k) acc[k] += t[u][k];
  }
  if (j >= P.n) return;
  // amp2 first, then the power-of-two column scale: the same bits as one
  // multiplication by amp2 * colscale while both are normal, and no subnormal
  // factor for a column whose scale is near the bottom of the float range
  float res[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const float as = amp2 * acc[k];
    res[k] = colscale ? as * colscale[min(c0 + k, nrhs - 1)] : as;
  }
  // Y is read only when beta is nonzero (two loops, so that the load is not
  // speculated into the common beta = 0 case as an extra round trip)
  if (beta == 0.f) {
#pragma unroll
    for (int k = 0; k < KC; ++k)
      if (c0 + k < nrhs) Y[(size_t)(c0 + k) * ldy + dst] = res[k];
  } else {
#pragma unroll
    for (int k = 0; k < KC; ++k)
      if (c0 + k < nrhs) {
        float* y = Y + (size_t)(c0 + k) * ldy + dst;
        *y = res[k] + beta * *y;
      }
  }
}

template <int KC>
__global__ void reduce_kernel(const TilePlan P, int nrhs, const float* __restrict__ part, int pcols,
                              const float* __restrict__ colscale, float amp2, float* Y, int ldy, float beta,
                              CgGate gate) {
  reduce_body<KC>([&] { return gate.skip_all(); }, blockIdx.x, blockIdx.y, P, nrhs, part, pcols, colscale, amp2, Y, ldy,
              beta);
}

// ---------------------------------------------------------------- workspace

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
  b.part = cv.template take<float>((size_t)plan_slots(n) * nrhs * kRowTile);
}

size_t mfma_workspace(int n, int nrhs, int prec) {
  if (n <= 0 || nrhs <= 0) return 0;
  Sizer s;
  ProdBufs b;
  carve_prod(s, n, nrhs, prec, b);
  return s.used;
}

float plan_threshold(int prec) { return prec == GPL_PREC_F16X3 ? kSkipF16x3 : kSkipFp32; }
float plan_lo_threshold(int prec) { return prec == GPL_PREC_F16X3 ? kLoF16x3 : kSkipFp32; }

// ---------------------------------------------------------------- launches

template <int CB>
static void launch_f16x3(bool packed, const TilePlan& P, const _Float16* Vh, const _Float16* Vl, int ncp,
                         int ncols, float* part, int pcols, int c0, CgGate gate, hipStream_t stream) {
  if constexpr (CB == 4) {  // the chunk filter is built for the 64-column form only (elsewhere it is ignored)
    if (gate.chunk_gen && !packed) {
      hipLaunchKernelGGL((mvm_f16x3_kernel<4, false, true>), dim3(P.nw / kWaves), dim3(256), 0, stream, P, Vh, Vl,
                         ncp, ncols, part, pcols, c0, gate);
      return;
    }
  }
  if (packed)
    hipLaunchKernelGGL((mvm_f16x3_kernel<CB, true>), dim3(P.nw / kWaves), dim3(256), 0, stream, P, Vh, Vl, ncp,
                       ncols, part, pcols, c0, gate);
  else
    hipLaunchKernelGGL((mvm_f16x3_kernel<CB, false>), dim3(P.nw / kWaves), dim3(256), 0, stream, P, Vh, Vl, ncp,
                       ncols, part, pcols, c0, gate);
}

template <int CB>
static void launch_f32(const TilePlan& P, float s2, const float* Vp, int ncp, int ncols, float* part, int pcols,
                       int c0, CgGate gate, hipStream_t stream) {
  hipLaunchKernelGGL((mvm_f32_kernel<CB>), dim3(P.nw / kWaves), dim3(256), 0, stream, P, s2, Vp, ncp, ncols, part,
                     pcols, c0, gate);
}

int mfma_carve(const TilePlan& P, int prec, int nrhs, void* ws, size_t ws_bytes, ProdBufs& b) {
  GPL_TRY(check_ws(ws, ws_bytes, mfma_workspace(P.n, nrhs, prec)));
  Carver cv(ws, ws_bytes);
  carve_prod(cv, P.n, nrhs, prec, b);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  return GPL_OK;
}

__global__ void zero_words_kernel(unsigned* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

static int zero_words(void* p, size_t words, hipStream_t stream) {
  const int blocks = (int)std::min<size_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_words_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, stream, static_cast<unsigned*>(p),
                     words);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int mfma_zero_rhs(const ProdBufs& b, int prec, hipStream_t stream) {
  const size_t elems = (size_t)b.ncp * b.ldh;  // ldh is a multiple of 64: whole words
  if (prec == GPL_PREC_F16X3) {
    GPL_TRY(zero_words(b.Vh, elems / 2, stream));
    return zero_words(b.Vl, elems / 2, stream);
  }
  return zero_words(b.Vp, elems, stream);
}

int mfma_prep_rhs(const TilePlan& P, const ProdBufs& b, int prec, int nrhs, const float* V, int ldv, CgGate gate,
                  hipStream_t stream) {
  const int n = P.n;
  if (prec == GPL_PREC_F16X3) {
    hipLaunchKernelGGL(colmax_kernel, dim3(kColmaxBlocks, nrhs), dim3(256), 0, stream, n, V, ldv, b.colmax, gate);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(split_rhs_kernel, dim3(cdiv(b.ldh, 256), b.ncp), dim3(256), 0, stream, n, nrhs, V, ldv, P.perm,
                       b.colmax, b.Vh, b.Vl, b.ldh, b.ncp, b.inv_scale, gate);
  } else {
    hipLaunchKernelGGL(pack_rhs_kernel, dim3(cdiv(b.ldh, 256), b.ncp), dim3(256), 0, stream, n, nrhs, V, ldv, P.perm,
                       b.Vp, b.ldh, b.ncp, gate);
  }
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int mfma_product(const TilePlan& P, const ProdBufs& b, int prec, float s2, float amp2, int nrhs, float* Y, int ldy,
                 float beta, CgGate gate, hipStream_t stream) {
  const bool f16 = prec == GPL_PREC_F16X3;
  // column blocks of up to 64 columns per pass; each pass writes its own columns
  for (int c0 = 0; c0 < b.ncp; c0 += kMaxCB * 16) {
    const int cb = std::min(kMaxCB, (b.ncp - c0) / 16);
    const int ncols = std::min(nrhs - c0, cb * 16);
    hipEvent_t t0 = timing_begin(stream);
    if (f16) {
      // columns c0.. of each chunk (rhs_at layout); the pass with the last block
      // may have it packed
      const _Float16* vh = b.Vh + (size_t)c0 * kChunk;
      const _Float16* vl = b.Vl + (size_t)c0 * kChunk;
      const bool pk = c0 + cb * 16 >= nrhs && last_block_packed(nrhs);
      switch (cb) {
        case 4: launch_f16x3<4>(pk, P, vh, vl, b.ncp, ncols, b.part, nrhs, c0, gate, stream); break;
        case 3: launch_f16x3<3>(pk, P, vh, vl, b.ncp, ncols, b.part, nrhs, c0, gate, stream); break;
        case 2: launch_f16x3<2>(pk, P, vh, vl, b.ncp, ncols, b.part, nrhs, c0, gate, stream); break;
        default: launch_f16x3<1>(pk, P, vh, vl, b.ncp, ncols, b.part, nrhs, c0, gate, stream); break;
      }
    } else {
      const float* vp = b.Vp + (size_t)c0 * kChunk;
      switch (cb) {
        case 4: launch_f32<4>(P, s2, vp, b.ncp, ncols, b.part, nrhs, c0, gate, stream); break;
        case 3: launch_f32<3>(P, s2, vp, b.ncp, ncols, b.part, nrhs, c0, gate, stream); break;
        case 2: launch_f32<2>(P, s2, vp, b.ncp, ncols, b.part, nrhs, c0, gate, stream); break;
        default: launch_f32<1>(P, s2, vp, b.ncp, ncols, b.part, nrhs, c0, gate, stream); break;
      }
    }
    GPL_LAUNCH_CHECK();
    timing_end(t0, stream);
  }
  // four columns a thread when that still leaves sixteen workgroups per compute
  // unit (measured: 64 columns at N = 160k 33.6 against 38.8 us with one column
  // a thread; at N = 40k, where that gives ten, 24.5 against 22.9 us)
  const bool wide = (long)cdiv(P.n, 256) * cdiv(nrhs, 4) >= 16L * (P.wround / kWaves);
  hipLaunchKernelGGL(wide ? reduce_kernel<4> : reduce_kernel<1>, dim3(cdiv(P.n, 256), cdiv(nrhs, wide ? 4 : 1)),
                     dim3(256), 0, stream, P, nrhs, b.part, nrhs, f16 ? b.inv_scale : nullptr, amp2, Y, ldy, beta,
                     gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

// ---------------------------------------------------------------- grouped launches (serving)
// One launch per stage over all slots of a batch; each slot uses up to 2 column
// blocks (32 right-hand sides), its own tile plan and its own buffers, so its
// result does not depend on the other slots. The slot's RHS block is written by
// the grouped PSF adjoint.

// The grouped kernel holds every wave variant, so its register count is their
// union; three waves per SIMD (at most 168 VGPRs) are asked for explicitly, as
// a batch of slots usually has more waves than the SIMDs hold at once.
__global__ __launch_bounds__(256, 3) void mvm_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  const int w = (blockIdx.x - B.off[s]) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  auto skip = [&] { return S.n_active[p] == 0; };
  if (S.prec == GPL_PREC_F16X3) {
    const bool pk = last_block_packed(S.nrhs);
    if (S.nrhs > 16) {
      if (pk) mvm_f16x3_wave<2, true>(skip, w, S.plan, S.Vh, S.Vl, S.ncp, S.nrhs, S.part, S.nrhs, 0);
      else mvm_f16x3_wave<2, false>(skip, w, S.plan, S.Vh, S.Vl, S.ncp, S.nrhs, S.part, S.nrhs, 0);
    } else {
      if (pk) mvm_f16x3_wave<1, true>(skip, w, S.plan, S.Vh, S.Vl, S.ncp, S.nrhs, S.part, S.nrhs, 0);
      else mvm_f16x3_wave<1, false>(skip, w, S.plan, S.Vh, S.Vl, S.ncp, S.nrhs, S.part, S.nrhs, 0);
    }
  } else {
    if (S.nrhs > 16)
      mvm_f32_wave<2>(skip, w, S.plan, S.s2, S.Vp, S.ncp, S.nrhs, S.part, S.nrhs, 0);
    else
      mvm_f32_wave<1>(skip, w, S.plan, S.s2, S.Vp, S.ncp, S.nrhs, S.part, S.nrhs, 0);
  }
}

__global__ void reduce_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  const int local = blockIdx.x - B.off[s];
  const int per = cdiv(S.N, 256);
  reduce_body<1>([&] { return S.n_active[p] == 0; }, local % per, local / per, S.plan, S.nrhs, S.part, S.nrhs,
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
  hipEvent_t t0 = timing_begin(stream);
  GPL_TRY(launch_grouped(mvm_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return S.plan.nw / kWaves; }, stream));
  timing_end(t0, stream);
  GPL_TRY(launch_grouped(reduce_grouped_kernel, hslots, dslots, nslots, p,
                         [](const ServeSlotDev& S) { return cdiv(S.N, 256) * S.nrhs; }, stream));
  return GPL_OK;
}

}  // namespace gpl
