// Low-rank preconditioner of A = B K B^T + sigma^2 I and the preconditioned CG
// that uses it: the GPyTorch scheme Sec. 3.3 cites for CG solves and the
// stochastic log-determinant (Gardner et al. 2018), which lowers the noise of
// that estimate (the reason Sec. 3.3 gives for avoiding it).
//
// Build. A partial pivoted Cholesky factor L (n x k, FP64) of M = B K B^T, its
// columns taken 64 at a time: the 64 largest remaining diagonal entries of
// M - L L^T are the candidates; their columns of M come from one application of
// B K B^T to unit vectors (the matrix-free product), minus L L^T on them
// (split-K rocBLAS dgemm); one four-wave workgroup runs a pivoted Cholesky on
// the 64 x 64 residual block (largest remaining diagonal first, stopping below
// a relative threshold), and the block's columns of L follow by a row-parallel
// triangular solve. Candidates the block does not take leave zero columns,
// which change neither L L^T nor the determinant identity below. With
//   G = sigma^2 I_k + L^T L,
//   ln|P| = (n - k) ln sigma^2 + ln|G|,  P = L L^T + sigma^2 I_n,
// G^{-1} and ln|G| are built by bordering in 64 x 64 blocks (Schur
// complements, their Cholesky factors and inverses) on a second stream: as soon
// as a block of L is in, its rows of L^T L and its bordering step run there
// while the caller's stream builds the next block.
// Solve. Preconditioned CG, one recurrence per column, with
//   P^{-1} v = (v - L G^{-1} L^T v) / sigma^2 (dgemm, dsymm, dgemm),
// FP32 vectors, FP64 scalars and Woodbury products; the alpha/beta of the
// first steps give the Lanczos tridiagonal of P^{-1/2} A P^{-1/2} with the
// usual CG formulas, and rz0 = b^T P^{-1} b is each probe's quadrature weight.
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "dense.hpp"
#include "internal.hpp"

namespace gpl {

constexpr int kPcBlock = 64;   // pivots per block
constexpr int kSideEvery = 2;  // blocks of the factor per event towards the side stream
constexpr int kPcSplits = 16;  // most splits of the reduction of a product with the factor
// A residual pivot below this share of the largest diagonal entry of M is not
// taken: the columns of M come from FP32 products (relative error ~5e-7), so
// smaller residuals are rounding noise, and at the workloads' noise level
// (sigma^2 ~ 6e-3 of the largest diagonal entry) they are far below what the
// preconditioner needs to capture.
constexpr double kPcRelTol = 1e-5;

// ---------------------------------------------------------------- diagonal of B K B^T

// d[I] = sum_{f, g in fp(I)} b_f b_g K(p_f, p_g) with b = B^T e_I: the fine
// points within the composite filter's reach of pixel I (weights
// g[ty] g[tx] / ss^2, zero outside the grid). One workgroup per pixel; the
// footprint is staged in LDS and the pair sum is reduced in a fixed order.
constexpr int kMaxFoot = (2 * GPL_PSF_MAX_RADIUS + 8) * (2 * GPL_PSF_MAX_RADIUS + 8);
__global__ __launch_bounds__(256) void bkb_diag_kernel(int n, int ss, const Taps taps, float s2, double amp2,
                                                       const float* __restrict__ px, const float* __restrict__ py,
                                                       double* d) {
  __shared__ float fx[kMaxFoot], fy[kMaxFoot], fw[kMaxFoot];
  __shared__ double red[4];
  __shared__ int s_cnt;
  const int I = blockIdx.x, iy = I / n, ix = I - iy * n, M = n * ss, L = taps.L, r = taps.r;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  // compact the in-grid footprint in a fixed (row-major) order
  if (threadIdx.x == 0) {
    int c = 0;
    const float inv = 1.f / (float)(ss * ss);
    for (int ty = 0; ty < L; ++ty) {
      const int gy = iy * ss + ty - r;
      if (gy < 0 || gy >= M) continue;
      for (int tx = 0; tx < L; ++tx) {
        const int gx = ix * ss + tx - r;
        if (gx < 0 || gx >= M) continue;
        const int j = gy * M + gx;
        fx[c] = px[j];
        fy[c] = py[j];
        fw[c] = taps.g[ty] * taps.g[tx] * inv;
        ++c;
      }
    }
    s_cnt = c;
  }
  __syncthreads();
  const int c = s_cnt;
  double s = 0.0;
  for (int e = threadIdx.x; e < c * c; e += blockDim.x) {
    const int a = e / c, b = e - a * c;
    const float dx = fx[a] - fx[b], dy = fy[a] - fy[b];
    s += (double)fw[a] * (double)fw[b] * (double)exp2_fast(-(fmaf(dx, dx, dy * dy) * s2));
  }
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) d[I] = amp2 * s;
}

// ---------------------------------------------------------------- candidate selection

// Exclusive prefix sum of v over the workgroup in thread order (wave scans by
// lane shuffles, then one combine of the wave totals through LDS); *total gets
// the sum. Every thread of the workgroup must call it.
__device__ __forceinline__ int block_excl_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, tot = 0;
  for (int u = 0; u < nw; ++u) {
    const int c = wsum[u];
    tot += c;
    before += u < w ? c : 0;
  }
  __syncthreads();  // wsum may be reused
  *total = tot;
  return before + x - v;
}

// The kPcBlock largest positive entries of d (ranked by their FP32 value, ties
// by lower index), in index order, into cand[0..kPcBlock); missing slots get
// -1. One workgroup: a three-pass radix select on the FP32 bit patterns (11, 11
// and 10 bits; each pass a histogram of the keys that match the prefix so far,
// and a top-down scan of the bins for the one where the count reaches the
// number still needed), then an ordered compaction.
constexpr int kSelThreads = 1024;
constexpr int kSelCache = 16;  // keys a thread keeps in registers (n up to 16384)
constexpr int kBinsPer = 2048 / kSelThreads;  // histogram bins per thread in the scans
static_assert(kBinsPer * kSelThreads == 2048, "the threads cover the 2048 bins of a pass");
__global__ __launch_bounds__(kSelThreads) void select_top_kernel(int n, const double* __restrict__ d, int* cand) {
  __shared__ int hist[2048];
  __shared__ int wsum[kSelThreads / 64];
  __shared__ unsigned s_prefix, s_mask;
  __shared__ int s_need, s_bin, s_above;
  const int t = threadIdx.x;
  auto key = [&](int i) -> unsigned {
    const double v = d[i];
    return v > 0.0 ? __float_as_uint((float)v) : 0u;
  };
  // thread t takes the index range [i0, i1) in every pass; with at most
  // kSelCache indices a thread, their keys are loaded once, all together, and
  // kept in registers (a loop of loads and LDS atomics would wait on each load)
  const int per = cdiv(n, kSelThreads), i0 = min(n, t * per), i1 = min(n, i0 + per);
  const bool cached = per <= kSelCache;
  unsigned kc[kSelCache];
  if (cached) {
#pragma unroll
    for (int e = 0; e < kSelCache; ++e) {
      const double v = d[min(i0 + e, n - 1)];
      kc[e] = (i0 + e < i1 && v > 0.0) ? __float_as_uint((float)v) : 0u;
    }
  }
  if (t == 0) {
    s_prefix = 0u;
    s_mask = 0u;
    s_need = kPcBlock;
  }
  const int shifts[3] = {21, 10, 0}, widths[3] = {11, 11, 10};
  for (int pass = 0; pass < 3; ++pass) {
    const int sh = shifts[pass], nb = 1 << widths[pass];
    for (int q = t; q < nb; q += kSelThreads) hist[q] = 0;
    __syncthreads();
    const unsigned prefix = s_prefix, mask = s_mask;
    const int need = s_need;
    if (cached) {
#pragma unroll
      for (int e = 0; e < kSelCache; ++e) {
        const unsigned k = kc[e];
        if (k != 0u && (k & mask) == prefix) atomicAdd(&hist[(k >> sh) & (nb - 1)], 1);
      }
    } else {
      for (int i = i0; i < i1; ++i) {
        const unsigned k = key(i);
        if (k != 0u && (k & mask) == prefix) atomicAdd(&hist[(k >> sh) & (nb - 1)], 1);
      }
    }
    __syncthreads();
    // thread t covers bins nb-1-kBinsPer*t-j, j < kBinsPer (top down); the
    // chosen bin is the highest whose count from the top reaches `need`, else
    // bin 0 with everything above it
    int h[kBinsPer], mine = 0;
#pragma unroll
    for (int j = 0; j < kBinsPer; ++j) {
      const int bj = nb - 1 - kBinsPer * t - j;
      h[j] = bj >= 0 ? hist[bj] : 0;
      mine += h[j];
    }
    int total;
    int run = block_excl_scan(mine, wsum, &total);
    if (t == 0) {
      s_bin = 0;
      s_above = total - hist[0];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBinsPer; ++j) {
      if (run < need && need <= run + h[j]) {
        s_bin = nb - 1 - kBinsPer * t - j;
        s_above = run;
      }
      run += h[j];
    }
    __syncthreads();
    if (t == 0) {
      s_need = need - s_above;
      s_prefix = prefix | ((unsigned)s_bin << sh);
      s_mask = mask | ((unsigned)(nb - 1) << sh);
    }
    __syncthreads();
  }
  // threshold key T = s_prefix: every key > T is taken, and the s_need lowest
  // indices with key == T (fewer if there are not that many); thread t scans
  // the index range [i0, i1) so that positions follow index order
  const unsigned T = s_prefix;
  const int eq_take = s_need;
  int above = 0, equal = 0;
  if (cached) {
#pragma unroll
    for (int e = 0; e < kSelCache; ++e) {
      const unsigned k = kc[e];  // 0 past i1
      above += (k != 0u && k > T);
      equal += (k != 0u && k == T);
    }
  } else {
    for (int i = i0; i < i1; ++i) {
      const unsigned k = key(i);
      above += (k != 0u && k > T);
      equal += (k != 0u && k == T);
    }
  }
  int tot_eq;
  int eq_before = block_excl_scan(equal, wsum, &tot_eq);
  const int mine = above + max(0, min(equal, eq_take - eq_before));
  int total;
  int pos = block_excl_scan(mine, wsum, &total);
  auto emit = [&](int i, unsigned k) {
    bool take = false;
    if (k != 0u && k > T) {
      take = true;
    } else if (k != 0u && k == T) {
      take = eq_before < eq_take;
      ++eq_before;
    }
    if (take && pos < kPcBlock) cand[pos++] = i;
  };
  if (cached) {
#pragma unroll
    for (int e = 0; e < kSelCache; ++e)
      if (i0 + e < i1) emit(i0 + e, kc[e]);
  } else {
    for (int i = i0; i < i1; ++i) emit(i, key(i));
  }
  for (int q = total + t; q < kPcBlock; q += kSelThreads) cand[q] = -1;
}

// ---------------------------------------------------------------- small element-wise kernels

// The product's right-hand side for the unit pixel columns, written straight
// into its buffers (the product then runs on them as prepared): column c is
// B^T e_{cand[c]}, the composite filter's footprint g(fx - ss Ix) g(fy - ss Iy)
// / ss^2 around that pixel, formed with the FP32 operations the general adjoint
// applies to it and placed at the sorted positions of the product's plan. The
// footprint of the previous block's candidate prev[c] is cleared first (the
// buffers hold nothing else: they were zeroed when the product was prepared).
// The precision form scales column c by 2^e from the bound max |B^T e| <= 1 /
// ss^2 (non-negative taps summing to one) and splits it into FP16 hi (nearest)
// and lo, as the CG loop's fused adjoint does. One workgroup per column.
__global__ __launch_bounds__(256) void unit_rhs_kernel(int n, int ss, const Taps taps, const int* cand, int* prev,
                                                       RhsOut o, int* chunk_gen, int gen) {
  const int c = blockIdx.x;
  const int M = n * ss, L = taps.L, r = taps.r;
  const bool f16 = o.prec == GPL_PREC_F16X3;
  const int hs = hi_slot(c, o.nrhs);
  const bool packed = last_block_packed(o.nrhs) && c >= packed_block_start(o.nrhs);
  const float inv_ss2 = 1.f / (float)(ss * ss);
  float scale = 1.f;
  if (f16) {
    const int e = min(14 - ilogbf(inv_ss2) - 1, 126);  // bound * 2^e in [2^13, 2^14)
    scale = ldexpf(1.f, e);
    if (threadIdx.x == 0) o.inv_scale[c] = ldexpf(1.f, -e) / 2048.f;  // with the 2^11 of the exp tile
  }
  auto put = [&](int j, float v) {
    if (f16) {
      const size_t at = rhs_at(hs, j, o.ncp);
      const float sv = v * scale;
      const _Float16 h = (_Float16)sv;
      const _Float16 l = (_Float16)(sv - (float)h);
      o.Vh[at] = h;
      if (packed) o.Vh[at + kChunk] = l;  // slot hs + 1 of the same chunk
      else o.Vl[at] = l;
    } else {
      o.Vp[rhs_at(c, j, o.ncp)] = v;
    }
  };
  // the footprint of pixel I: fine point (ss Iy + ty - r, ss Ix + tx - r) has weight g[ty] g[tx] / ss^2
  auto footprint = [&](int I, bool zero) {
    const int Iy = I / n, Ix = I - Iy * n;
    for (int t = threadIdx.x; t < L * L; t += blockDim.x) {
      const int ty = t / L, tx = t - ty * L;
      const int fy = ss * Iy + ty - r, fx = ss * Ix + tx - r;
      if (fy < 0 || fy >= M || fx < 0 || fx >= M) continue;
      const int j = o.irank[fy * M + fx];
      put(j, zero ? 0.f : (taps.g[ty] * taps.g[tx]) * inv_ss2);
      if (!zero) chunk_gen[j / kChunk] = gen;  // the product evaluates this chunk
    }
  };
  const int old = prev[c], now = cand[c];
  if (old >= 0) footprint(old, true);
  __syncthreads();  // a footprint shared by both is written after it was cleared
  if (now >= 0) footprint(now, false);
  if (threadIdx.x == 0) prev[c] = now;
}

// Ct (FP64, kPcBlock x npix, ld kPcBlock: the residual block stored by pixel
// rows) = Mc^T (Mc FP32, npix x kPcBlock, ld npix). Thread (c, i) with c the
// fastest index, so that the stores are contiguous.
__global__ void widen_kernel(int npix, const float* __restrict__ Mc, double* Ct) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = e % kPcBlock, i = e / kPcBlock;
  if (i < npix) Ct[e] = (double)Mc[(size_t)c * npix + i];
}

// Lc (kPcBlock x j) = L[cand, 0..j): rows of the factor at the candidates (0 for
// a missing candidate).
__global__ void gather_rows_kernel(int j, const double* __restrict__ L, int ldl, const int* cand, double* Lc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kPcBlock * j) return;
  const int c = q % kPcBlock, col = q / kPcBlock;
  Lc[(size_t)col * kPcBlock + c] = cand[c] >= 0 ? L[(size_t)col * ldl + cand[c]] : 0.0;
}

// Pivoted Cholesky of the residual block S = C[cand, :] (kPcBlock x kPcBlock;
// C, the npix x kPcBlock residual columns, is stored by pixel rows in Ct)
// by four waves: lane a of every wave owns candidate a, and wave q holds the
// entries (a, b) of its quarter of the columns b in registers. Every wave also
// keeps the residual diagonal (lane a: entry (a, a)) and finds each step's
// pivot itself: the largest remaining diagonal entry (lowest candidate index on
// ties), while it exceeds tol (a share of the largest diagonal entry of M,
// dmax[0]). The wave holding column p forms l = S[:, p] / sqrt(S[p][p]) (the
// reciprocal square root refined to FP64 accuracy) and publishes it in LDS; after one barrier every wave applies S -= l l^T to its
// registers and to its copy of the diagonal (l is double-buffered by step
// parity, so one barrier per step suffices). Outputs order[0..kPcBlock) (taken
// candidates in pivot order first, then the rest), *taken, and R (kPcBlock x
// kPcBlock, lower, R[u][v] = l of step v at the u-th pivot; identity on the
// untaken part).
constexpr int kPivWaves = 4;
constexpr int kPivCols = kPcBlock / kPivWaves;

// A 64-bit value of another lane of the same row of 16 lanes (DPP control CTRL).
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long k) {
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)k, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(k >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)hi << 32) | lo;
}

// Largest 64-bit key of the wave (every lane active), in every lane: the
// maximum within each row of 16 lanes by DPP (exchanges inside quads, then
// rotations of the row by 4 and 8 lanes), then the four row maxima as scalars.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
  unsigned long long o;
  o = dpp_u64<0xB1>(k);  // quad_perm [1, 0, 3, 2]
  k = o > k ? o : k;
  o = dpp_u64<0x4E>(k);  // quad_perm [2, 3, 0, 1]
  k = o > k ? o : k;
  o = dpp_u64<0x124>(k);  // row_ror:4
  k = o > k ? o : k;
  o = dpp_u64<0x128>(k);  // row_ror:8
  k = o > k ? o : k;
  unsigned long long m = 0ull;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)k, 16 * r);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(k >> 32), 16 * r);
    const unsigned long long x = ((unsigned long long)hi << 32) | lo;
    m = x > m ? x : m;
  }
  return m;
}

__global__ __launch_bounds__(64 * kPivWaves) void block_pivot_kernel(const double* __restrict__ Ct, int npix,
                                                                     const int* cand, const double* dmax,
                                                                     double rel_tol, int* order, int* taken,
                                                                     double* R) {
  __shared__ double lv[kPcBlock][kPcBlock];  // lv[step][a]: l of each step
  __shared__ double lc[2][kPcBlock];         // l with the pivot's and used entries zeroed
  __shared__ int s_perm[kPcBlock];
  // the wave index as a scalar: the owner wave then picks its entry of column p
  // by a register-relative move instead of a chain of selects
  const int a = threadIdx.x & 63, q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b0 = q * kPivCols;
  const int ca = cand[a];
  // every load at a valid address (row 0 for a missing candidate) and issued
  // together; a missing candidate's entries are zeroed afterwards (a load under
  // a condition would be branched around and waited for on its own)
  int cb[kPivCols];
#pragma unroll
  for (int u = 0; u < kPivCols; ++u) cb[u] = cand[b0 + u];
  const double* crow = Ct + (size_t)max(ca, 0) * kPcBlock;
  double s[kPivCols];  // s[u] = entry (a, b0 + u)
#pragma unroll
  for (int u = 0; u < kPivCols; ++u) s[u] = crow[b0 + u];
  double dg = crow[a];  // entry (a, a)
#pragma unroll
  for (int u = 0; u < kPivCols; ++u) s[u] = (ca >= 0 && cb[u] >= 0) ? s[u] : 0.0;
  dg = ca >= 0 ? dg : 0.0;
  bool used = ca < 0, piv = false;
  const double tol = rel_tol * dmax[0];
  int cnt = 0;
  for (int step = 0; step < kPcBlock; ++step) {
    // wave argmax of the remaining diagonal, lowest index on ties: positive
    // doubles order as their bit patterns; entries <= 0 never exceed tol >= 0
    const unsigned long long key = (!used && dg > 0.0) ? (unsigned long long)__double_as_longlong(dg) : 0ull;
    const unsigned long long kmax = wave_max_u64(key);
    const double v = __longlong_as_double((long long)kmax);
    if (!(v > tol)) break;
    const int p = __ffsll((unsigned long long)__ballot(key == kmax)) - 1;
    const int buf = step & 1;
    if (q == p / kPivCols) {  // this wave holds column p
      const double sp = s[p - b0];
      const double r = rsqrt_f64(v), lpp = v * r;
      const double l = a == p ? lpp : (used ? 0.0 : sp * r);
      lv[step][a] = l;
      lc[buf][a] = (a == p || used) ? 0.0 : l;
      if (a == 0) s_perm[step] = p;
    }
    __syncthreads();
    {  // la = 0 at the pivot and the used rows: their entries stay as they are
      const double la = lc[buf][a];
#pragma unroll
      for (int u = 0; u < kPivCols; ++u) s[u] -= la * lc[buf][b0 + u];
      dg -= la * la;
    }
    used = used || a == p;
    piv = piv || a == p;
    cnt = step + 1;
  }
  // order: taken pivots first (pivot order), then the rest in candidate order
  const unsigned long long rest = __ballot(!piv);
  if (q == 0) {
    if (a < cnt) order[a] = s_perm[a];
    if (!piv) order[cnt + __popcll(rest & ((1ull << a) - 1ull))] = a;
    if (a == 0) *taken = cnt;
  }
  // R[u][v] = lv[v][perm[u]] for v <= u < cnt; identity beyond (column a = v)
  const int vcol = a;
#pragma unroll
  for (int k = 0; k < kPivCols; ++k) {
    const int u = b0 + k;
    double val = 0.0;
    if (u < cnt && vcol < cnt) val = vcol <= u ? lv[vcol][s_perm[u]] : 0.0;
    else if (u == vcol) val = 1.0;
    R[(size_t)vcol * kPcBlock + u] = val;
  }
}

// The block's new columns of L and the residual diagonal, four lanes per pixel
// row i (each holding 16 of the 64 entries):
//   x[u] = C[i, order[u]] for u < taken (0 beyond), then x R^{-T}: forward
//   substitution taken column by column, so that the updates of a row's
//   remaining entries are independent (each entry still receives its updates
//   in the same order as in the row-by-row form);
//   rows that a pivoted Cholesky fixes exactly: zero at the pivots of earlier
//   blocks (their residual is zero; the computed one is rounding noise that
//   the solve would amplify), and R's row u at the block's u-th pivot (the
//   computed columns of M are not exactly symmetric, so the solve alone would
//   not return it);
//   d -= sum_u x[u]^2 (each lane's 16 in u order, then the quad in a fixed
//   order), clamped at 0, exactly 0 at the new pivots,
//   which are marked in is_piv; pivots[j0 + u] = the pixel of pivot u (-1 where
//   none was taken).
constexpr int kNcPix = 64;  // pixels per workgroup of the new-columns kernel, four lanes each
__global__ __launch_bounds__(256) void new_columns_kernel(int npix, const double* __restrict__ Ct,
                                                          const int* order, const int* taken,
                                                          const double* __restrict__ R, const int* cand, double* d,
                                                          int* is_piv, double* __restrict__ Lnew, int ldl,
                                                          int* pivots, int j0) {
  __shared__ double Rz[kPcBlock][kPcBlock];       // Rz[v][w] = entry (w, v) of R for w > v, else 0
  __shared__ double rows[kNcPix][kPcBlock + 1];   // the workgroup's rows of the residual columns
  __shared__ double idg[kPcBlock], rdg[kPcBlock];  // 1 / R(v, v) and R(v, v)
  __shared__ int s_ord[kPcBlock], s_pix[kPcBlock];
  const int t = threadIdx.x;
  const int cnt = *taken;
  const int p0 = blockIdx.x * kNcPix;
  // the workgroup's rows are one contiguous stretch of Ct: coalesced loads, all
  // issued before the first LDS store (element t + 256 k is row t / 64 + 4k,
  // column t % 64; rows past npix read the last row)
  static_assert(kNcPix * kPcBlock == 16 * 256, "sixteen elements a thread");
  {
    double tmp[16];
    const int cc = t & (kPcBlock - 1), rb = t / kPcBlock;
#pragma unroll
    for (int k = 0; k < 16; ++k) tmp[k] = Ct[(size_t)min(p0 + rb + 4 * k, npix - 1) * kPcBlock + cc];
#pragma unroll
    for (int k = 0; k < 16; ++k) rows[rb + 4 * k][cc] = tmp[k];
  }
  for (int e = t; e < kPcBlock * kPcBlock; e += 256) {
    const int v = e / kPcBlock, w = e - v * kPcBlock;
    const double r = R[e];  // R is column-major: R[v * 64 + w] = entry (w, v)
    (&Rz[0][0])[e] = w > v ? r : 0.0;
    if (w == v) {
      idg[v] = 1.0 / r;
      rdg[v] = r;
    }
  }
  if (t < kPcBlock) {
    const int o = order[t];
    const int pix = t < cnt ? cand[o] : -1;
    s_ord[t] = o;
    s_pix[t] = pix;
    if (blockIdx.x == 0 && pivots) pivots[j0 + t] = pix;
  }
  __syncthreads();
  // pixel i = p0 + t / 4; lane sub = t % 4 of its quad holds x[16 sub .. 16 sub + 15].
  // Forward substitution x R = row (R upper triangular): at step v the owner
  // lane of x[v] scales it by 1 / R(v, v), the quad takes it by a DPP broadcast,
  // and every lane subtracts x[v] R(v, w) from its entries (zero for w <= v).
  const int pl = t >> 2, sub = t & 3, i = p0 + pl;
  double x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int u = 16 * sub + k;
    x[k] = u < cnt ? rows[pl][s_ord[u]] : 0.0;  // order[] is a permutation
  }
  // steps 16 ow .. 16 ow + 15, whose pivots lane ow holds (DPP quad_perm
  // [ow, ow, ow, ow] is the control 0x55 ow)
  auto steps = [&](auto owc) {
    constexpr int ow = decltype(owc)::value;
#pragma unroll
    for (int vv = 0; vv < 16; ++vv) {
      const int v = 16 * ow + vv;
      if (sub == ow) x[vv] *= idg[v];
      const unsigned long long xb = dpp_u64<0x55 * ow>((unsigned long long)__double_as_longlong(x[vv]));
      const double xv = __longlong_as_double((long long)xb);
      const double* rz = &Rz[v][16 * sub];
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = fma(-xv, rz[k], x[k]);
    }
  };
  steps(std::integral_constant<int, 0>{});
  steps(std::integral_constant<int, 1>{});
  steps(std::integral_constant<int, 2>{});
  steps(std::integral_constant<int, 3>{});
  int pu = -1;
#pragma unroll
  for (int u = 0; u < kPcBlock; ++u) pu = s_pix[u] == i ? u : pu;
  const int ic = min(i, npix - 1);
  if (is_piv[ic]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = 0.0;
  } else if (pu >= 0) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int u = 16 * sub + k;
      x[k] = u < cnt ? (u == pu ? rdg[u] : Rz[u][pu]) : 0.0;  // entry (pu, u) of R (zero for u > pu)
    }
  }
  double sq = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (16 * sub + k < cnt) sq = fma(x[k], x[k], sq);
  sq += __longlong_as_double((long long)dpp_u64<0xB1>((unsigned long long)__double_as_longlong(sq)));
  sq += __longlong_as_double((long long)dpp_u64<0x4E>((unsigned long long)__double_as_longlong(sq)));
  if (i >= npix) return;
  if (sub == 0) {
    double v = d[i] - sq;
    if (pu >= 0) {
      v = 0.0;
      is_piv[i] = 1;
    }
    d[i] = v > 0.0 ? v : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) Lnew[(size_t)(16 * sub + k) * ldl + i] = x[k];
}

__global__ void set_ints_kernel(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void zero_ints_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// dmax[0] = max d (one workgroup).
__global__ __launch_bounds__(1024) void dmax_kernel(int n, const double* d, double* dmax) {
  __shared__ double red[16];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, d[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    *dmax = r;
  }
}

// ln|P| = (n - k) ln s + ln|G|.
__global__ void logdet_p_kernel(int n, int k, double s, const double* logdet_g, double* out) {
  if (threadIdx.x == 0) *out = (double)(n - k) * log(s) + *logdet_g;
}

// ---------------------------------------------------------------- build workspace

struct PcBuf {
  float *T2, *Mc;
  double *C, *Lc, *R, *d, *dmax, *logdet_g, *split;
  double *Y, *W, *T, *Dinv, *ld_part, *split2;  // G and its bordered inverse (on the side stream)
  size_t split2_elems;
  size_t split_elems;  // doubles of split
  int *cand, *prev, *order, *taken, *info, *is_piv;
  int* chunk_gen;  // [chunks of the plan] the last block whose unit columns touch the chunk
  void* mvm_ws;
  size_t mvm_bytes;
  void *blas, *blas2;
};

template <class Cv>
static void carve_pc(Cv& c, int npix, int N, int k, int prec, PcBuf& b) {
  const int ldf = round_up(N, 64);
  b.T2 = c.template take<float>((size_t)ldf * kPcBlock);
  b.Mc = c.template take<float>((size_t)npix * kPcBlock);
  b.C = c.template take<double>((size_t)npix * kPcBlock);
  b.Lc = c.template take<double>((size_t)kPcBlock * std::max(k, 1));
  b.R = c.template take<double>((size_t)kPcBlock * kPcBlock);
  b.split_elems = split_gemm_scratch(npix, kPcBlock, kPcSplits) / sizeof(double);
  b.split = c.template take<double>(b.split_elems);
  b.d = c.template take<double>(npix);
  b.dmax = c.template take<double>(1);
  b.logdet_g = c.template take<double>(1);
  b.Y = c.template take<double>((size_t)kPcBlock * std::max(k, 1));
  b.W = c.template take<double>((size_t)kPcBlock * std::max(k, 1));
  b.T = c.template take<double>((size_t)kPcBlock * kPcBlock);
  b.Dinv = c.template take<double>((size_t)kPcBlock * kPcBlock);
  b.ld_part = c.template take<double>(std::max(k / kPcBlock, 1));
  b.split2_elems = split_gemm_scratch(kPcBlock, std::max(k, 1), kPcSplits) / sizeof(double);
  b.split2 = c.template take<double>(b.split2_elems);
  b.blas2 = c.template take<char>(kBlasScratch);
  b.cand = c.template take<int>(kPcBlock);
  b.prev = c.template take<int>(kPcBlock);
  b.order = c.template take<int>(kPcBlock);
  b.taken = c.template take<int>(1);
  b.info = c.template take<int>(1);
  b.is_piv = c.template take<int>(npix);
  b.chunk_gen = c.template take<int>((size_t)kChunksPerTile * cdiv(N, kRowTile));
  b.mvm_bytes = mvm_workspace(N, kPcBlock, prec);
  b.mvm_ws = c.template take<char>(b.mvm_bytes);
  b.blas = c.template take<char>(kBlasScratch);
}

static int check_pc_problem(const gpl_problem* prob, Taps& taps) {
  GPL_REQUIRE(prob != nullptr, "problem is NULL");
  const gpl_grid* g = &prob->grid;
  GPL_REQUIRE(g->n >= 1 && g->ss >= 1 && g->pix_scale > 0, "bad grid");
  GPL_REQUIRE(prob->px && prob->py, "problem points are NULL");
  GPL_REQUIRE(prob->noise_sigma > 0 && std::isfinite(prob->noise_sigma), "noise_sigma must be > 0");
  GPL_TRY(check_kernel(&prob->kernel));
  GPL_TRY(make_taps(g, &prob->psf, taps));
  GPL_REQUIRE((2 * taps.r + g->ss) * (2 * taps.r + g->ss) <= kMaxFoot, "PSF footprint too large");
  return GPL_OK;
}

// ---------------------------------------------------------------- preconditioned CG

struct PcgState {
  double rz;     // r . P^{-1} r of the current residual
  double rr;     // r . r of the current residual
  double alpha;  // alpha of the step that produced this state
  int active, iters, status, bad;
};

struct PcgBuf {
  float *R, *P, *AP, *T2, *Z;
  double *R64, *Z64, *W, *W2, *split;
  size_t split_elems;  // doubles of split
  int ldv, ldf;
  void* mvm_ws;
  size_t mvm_bytes;
  double *pap_part, *rr_part, *rz_part;
  int ntiles, nb;
  PcgState* st[2];
  double* bb;
  int* n_active;
  unsigned* pmax;
  void* blas;
};

template <class Cv>
static void carve_pcg(Cv& c, int npix, int N, int n, int ss, int k, int nrhs, int prec, PcgBuf& b) {
  b.ldv = round_up(npix, 64);
  b.ldf = round_up(N, 64);
  b.ntiles = psf_forward_tiles(n, ss);
  b.nb = cdiv(npix, 256);
  b.R = c.template take<float>((size_t)b.ldv * nrhs);
  b.P = c.template take<float>((size_t)b.ldv * nrhs);
  b.AP = c.template take<float>((size_t)b.ldv * nrhs);
  b.Z = c.template take<float>((size_t)b.ldv * nrhs);
  b.T2 = c.template take<float>((size_t)b.ldf * nrhs);
  b.R64 = c.template take<double>((size_t)b.ldv * nrhs);
  b.Z64 = c.template take<double>((size_t)b.ldv * nrhs);
  b.W = c.template take<double>((size_t)std::max(k, 1) * nrhs);
  b.W2 = c.template take<double>((size_t)std::max(k, 1) * nrhs);
  b.split_elems =
      std::max(split_gemm_scratch(nrhs, std::max(k, 1), kPcSplits), split_gemm_scratch(npix, nrhs, kPcSplits)) /
      sizeof(double);
  b.split = c.template take<double>(b.split_elems);
  b.mvm_bytes = mvm_workspace(N, nrhs, prec);
  b.mvm_ws = c.template take<char>(b.mvm_bytes);
  b.pap_part = c.template take<double>((size_t)b.ntiles * nrhs);
  b.rr_part = c.template take<double>((size_t)b.nb * nrhs);
  b.rz_part = c.template take<double>((size_t)b.nb * nrhs);
  b.st[0] = c.template take<PcgState>(nrhs);
  b.st[1] = c.template take<PcgState>(nrhs);
  b.bb = c.template take<double>(nrhs);
  b.n_active = c.template take<int>(2);
  b.pmax = c.template take<unsigned>((size_t)b.nb * nrhs);
  b.blas = c.template take<char>(kBlasScratch);
}

// Z64 = R64 = R (FP64 copies for the Woodbury products).
__global__ __launch_bounds__(256) void pcg_widen_kernel(int npix, const float* __restrict__ R, int ldv, double* R64,
                                                        double* Z64) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  const double v = R[(size_t)c * ldv + i];
  R64[(size_t)c * ldv + i] = v;
  Z64[(size_t)c * ldv + i] = v;
}

// P^{-1} R for every column: Wt = R64^T L (m x k); W2 = Wt G^{-1} (one
// symmetric product with the inverse the build left in G's lower triangle);
// Z64 = R64 - L W2^T. Both products with L have one short side (m columns)
// and run with their long reduction split. The caller finishes Z = Z64 / s.
static int woodbury(rocblas_handle h, int npix, int k, const double* L, int ldl, const double* Gi, int ldg, int nrhs,
                    const double* R64, double* Z64, int ldv, double* Wt, double* W2, double* split,
                    size_t split_elems, hipStream_t stream) {
  const double one = 1.0, zero = 0.0;
  GPL_TRY(split_gemm(h, rocblas_operation_transpose, rocblas_operation_none, nrhs, k, npix, kPcSplits, 1.0, R64, ldv,
                     L, ldl, 0.0, Wt, nrhs, split, split_elems, stream));
  if (rocblas_dsymm(h, rocblas_side_right, rocblas_fill_lower, nrhs, k, &one, Gi, ldg, Wt, nrhs, &zero, W2, nrhs) !=
      rocblas_status_success) {
    set_error("rocblas_dsymm (preconditioner) failed");
    return GPL_EHIP;
  }
  return split_gemm(h, rocblas_operation_none, rocblas_operation_transpose, npix, nrhs, k, kPcSplits, -1.0, L, ldl, W2,
                    nrhs, 1.0, Z64, ldv, split, split_elems, stream);
}

// Z = Z64 / s (FP32), partial r.z and (at init) partial |b|^2 and max |Z| per block.
__global__ __launch_bounds__(256) void pcg_zfinish_kernel(int npix, const double* __restrict__ Z64, int ldv,
                                                          double inv_s, const float* __restrict__ R, float* Z,
                                                          double* rz_part, int nb, const PcgState* st,
                                                          const int* n_active) {
  __shared__ double red[4];
  const int c = blockIdx.y;
  if (n_active && (*n_active == 0 || !st[c].active)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < npix) {
    const float z = (float)(Z64[(size_t)c * ldv + i] * inv_s);
    Z[(size_t)c * ldv + i] = z;
    s = (double)R[(size_t)c * ldv + i] * (double)z;
  }
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) rz_part[(size_t)c * nb + blockIdx.x] = s;
}

// R = B, X = 0, partial |b|^2.
__global__ __launch_bounds__(256) void pcg_init_kernel(int npix, const float* __restrict__ Bm, int ldb, float* X,
                                                       int ldx, float* R, int ldv, double* part, int nb) {
  __shared__ double red[4];
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < npix) {
    const float b = Bm[(size_t)c * ldb + i];
    R[(size_t)c * ldv + i] = b;
    X[(size_t)c * ldx + i] = 0.f;
    s = (double)b * b;
  }
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) part[(size_t)c * nb + blockIdx.x] = s;
}

// P = Z and partial max |P|, after the initial preconditioner application.
__global__ __launch_bounds__(256) void pcg_init_p_kernel(int npix, const float* __restrict__ Z, float* P, int ldv,
                                                         unsigned* pmax, int nb) {
  __shared__ float redm[4];
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float m = 0.f;
  if (i < npix) {
    const float z = Z[(size_t)c * ldv + i];
    P[(size_t)c * ldv + i] = z;
    m = fabsf(z);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) pmax[(size_t)c * nb + blockIdx.x] =
      __float_as_uint(fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3])));
}

// Initial state per column from the partials: rr = |b|^2, rz = b.P^{-1}b.
__global__ void pcg_init_state_kernel(int nrhs, const double* rr_part, const double* rz_part, int nb, PcgState* s0,
                                      PcgState* s1, double* bb, double* rz0, int* n_active, int limit) {
  __shared__ int count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < nrhs; c += blockDim.x) {
    double rr = 0.0, rz = 0.0;
    for (int b = 0; b < nb; ++b) {
      rr += rr_part[(size_t)c * nb + b];
      rz += rz_part[(size_t)c * nb + b];
    }
    PcgState z;
    z.rr = rr;
    z.rz = rz;
    z.alpha = 0.0;
    z.iters = 0;
    z.bad = 0;
    if (!isfinite(rr) || !isfinite(rz)) {
      z.status = GPL_CG_NONFINITE;
      z.active = 0;
    } else if (rr == 0.0 || limit == 0) {
      z.status = rr == 0.0 ? GPL_CG_CONVERGED : GPL_CG_MAXITER;
      z.active = 0;
    } else {
      z.status = GPL_CG_CONVERGED;
      z.active = 1;
    }
    s0[c] = z;
    s1[c] = z;
    bb[c] = rr;
    if (rz0) rz0[c] = rz;
    if (z.active) atomicAdd(&count, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    n_active[0] = count;
    n_active[1] = count;
  }
}

// alpha = rz / pAp; X += alpha P; R -= alpha AP; R64 = Z64 = R; partial r.r.
__global__ __launch_bounds__(256) void pcg_update1_kernel(int npix, float* X, int ldx, float* R, const float* P,
                                                          const float* AP, int ldv, double* R64, double* Z64,
                                                          const double* pap_part, int ntiles, double* rr_part, int nb,
                                                          const PcgState* sin, PcgState* sout,
                                                          const int* n_active_in, int* n_active_out) {
  __shared__ double red[4];
  __shared__ double s_alpha;
  __shared__ int s_ok;
  const int c = blockIdx.y, bx = blockIdx.x;
  if (bx == 0 && c == 0 && threadIdx.x == 0) *n_active_out = 0;
  if (*n_active_in == 0) return;
  const PcgState st = sin[c];
  if (!st.active) return;
  const int i = bx * blockDim.x + threadIdx.x;
  const size_t iv = (size_t)c * ldv + i;
  float xv = 0.f, pv = 0.f, apv = 0.f, rv = 0.f;
  if (i < npix) {
    xv = X[(size_t)c * ldx + i];
    pv = P[iv];
    apv = AP[iv];
    rv = R[iv];
  }
  const double pap = threadIdx.x < 64 ? wave_fold_sum(pap_part + (size_t)c * ntiles, ntiles) : 0.0;
  if (threadIdx.x == 0) {
    const double a = st.rz / pap;
    const int ok = (pap > 0.0) && isfinite(a);
    s_alpha = ok ? a : 0.0;
    s_ok = ok;
    if (bx == 0) {
      sout[c].alpha = s_alpha;
      sout[c].bad = ok ? 0 : (isfinite(pap) ? 1 : 2);
    }
  }
  __syncthreads();
  double s = 0.0;
  if (s_ok && i < npix) {
    const float af = (float)s_alpha;
    X[(size_t)c * ldx + i] = fmaf(af, pv, xv);
    const float r = fmaf(-af, apv, rv);
    R[iv] = r;
    R64[iv] = r;
    Z64[iv] = r;
    s = (double)r * r;
  }
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) rr_part[(size_t)c * nb + bx] = s;
}

// beta = rz_new / rz; P = Z + beta P; block 0 records the Lanczos coefficients
// and decides the column's status (stop on the recursive residual |r|/|b|).
__global__ __launch_bounds__(256) void pcg_update2_kernel(int npix, const float* Z, float* P, int ldv,
                                                          const double* rr_part, const double* rz_part, int nb,
                                                          const PcgState* sin, PcgState* sout, const double* bb,
                                                          const int* n_active_in, int* n_active_out, double tol,
                                                          int max_iter, int fixed_iters, int n_lanczos, double* ab,
                                                          unsigned* pmax) {
  __shared__ double s_beta;
  __shared__ int s_go;
  __shared__ float redm[4];
  const int c = blockIdx.y, bx = blockIdx.x;
  const PcgState st = sin[c];
  if (*n_active_in == 0 || !st.active) {
    if (bx == 0 && threadIdx.x == 0) sout[c] = st;
    return;
  }
  const int i = bx * blockDim.x + threadIdx.x;
  const size_t iv = (size_t)c * ldv + i;
  float zv = 0.f, pv = 0.f;
  if (i < npix) {
    zv = Z[iv];
    pv = P[iv];
  }
  double rr_new = 0.0, rz_new = 0.0;
  if (threadIdx.x < 64) {
    rr_new = wave_fold_sum(rr_part + (size_t)c * nb, nb);
    rz_new = wave_fold_sum(rz_part + (size_t)c * nb, nb);
  }
  if (threadIdx.x == 0) {
    const PcgState half = sout[c];
    const double beta = rz_new / st.rz;
    PcgState nx;
    nx.alpha = half.alpha;
    nx.bad = 0;
    nx.iters = st.iters;
    nx.rr = st.rr;
    nx.rz = st.rz;
    nx.status = GPL_CG_CONVERGED;
    nx.active = 0;
    int go = 0;
    if (half.bad) {
      nx.status = half.bad == 1 ? GPL_CG_BREAKDOWN : GPL_CG_NONFINITE;
    } else if (!isfinite(rr_new) || !isfinite(rz_new) || !isfinite(beta)) {
      nx.status = GPL_CG_NONFINITE;
      nx.iters = st.iters + 1;
    } else {
      go = 1;
      nx.rr = rr_new;
      nx.rz = rz_new;
      nx.iters = st.iters + 1;
      if (bx == 0 && st.iters < n_lanczos) {
        double* e = ab + ((size_t)c * n_lanczos + st.iters) * 2;
        e[0] = half.alpha;
        e[1] = beta;
      }
      if (fixed_iters > 0) {
        nx.active = nx.iters < fixed_iters;
      } else if (sqrt(rr_new) <= tol * sqrt(bb[c])) {
        nx.active = 0;
      } else if (nx.iters >= max_iter) {
        nx.status = GPL_CG_MAXITER;
      } else {
        nx.active = 1;
      }
    }
    s_beta = beta;
    s_go = go;
    if (bx == 0) {
      sout[c] = nx;
      if (nx.active) atomicAdd(n_active_out, 1);
    }
  }
  __syncthreads();
  if (!s_go) return;
  float m = 0.f;
  if (i < npix) {
    const float pn = fmaf((float)s_beta, pv, zv);
    P[iv] = pn;
    m = fabsf(pn);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    pmax[(size_t)c * nb + bx] = __float_as_uint(fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3])));
}

__global__ void pcg_finalize_kernel(int nrhs, const PcgState* st, const double* bb, int* iters, double* relres,
                                    int* status, int n_lanczos, double* ab) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const PcgState s = st[c];
  if (iters) iters[c] = s.iters;
  if (relres) relres[c] = bb[c] > 0.0 ? sqrt(s.rr / bb[c]) : 0.0;
  if (status) status[c] = s.active ? GPL_CG_MAXITER : s.status;
  if (ab)
    for (int k = s.iters; k < n_lanczos; ++k) {
      ab[((size_t)c * n_lanczos + k) * 2 + 0] = 0.0;
      ab[((size_t)c * n_lanczos + k) * 2 + 1] = 0.0;
    }
}

__global__ void pcg_snapshot_kernel(const int* n_active, volatile int* host_flag) {
  if (threadIdx.x == 0) {
    *host_flag = *n_active;
    __threadfence_system();
  }
}

// Partial |b - A x|^2 per block and its fold (the true residual at exit).
__global__ __launch_bounds__(256) void pcg_true_residual_kernel(int npix, const float* __restrict__ Bm, int ldb,
                                                                const float* __restrict__ AX, int ldv, double* part,
                                                                int nb) {
  __shared__ double red[4];
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < npix) {
    const double d = (double)Bm[(size_t)c * ldb + i] - (double)AX[(size_t)c * ldv + i];
    s = d * d;
  }
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) part[(size_t)c * nb + blockIdx.x] = s;
}

__global__ void pcg_true_residual_fold_kernel(int nrhs, const double* part, int nb, const double* bb, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)c * nb + b];
  out[c] = bb[c] > 0.0 ? sqrt(s / bb[c]) : sqrt(s);
}

__global__ __launch_bounds__(256) void pcg_absmax_kernel(int npix, const float* __restrict__ X, int ldx,
                                                         unsigned* pmax, int nb) {
  __shared__ float redm[4];
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float m = i < npix ? fabsf(X[(size_t)c * ldx + i]) : 0.f;
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    pmax[(size_t)c * nb + blockIdx.x] = __float_as_uint(fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3])));
}

// Probe block Z = L g + sqrt(s) h (FP32 output), FP64 accumulation.
__global__ void probe_finish_kernel(int npix, const double* __restrict__ Lg, double sq, const float* __restrict__ h,
                                    int ldh, float* Z, int ldz) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npix) Z[(size_t)c * ldz + i] = (float)(Lg[(size_t)c * npix + i] + sq * (double)h[(size_t)c * ldh + i]);
}

struct PollFlags {
  int* flags = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int device = -1;
};

static int pcg_poll(PollFlags*& out) {
  thread_local PollFlags f;
  int dev = 0;
  GPL_HIP(hipGetDevice(&dev));
  if (f.flags == nullptr || f.device != dev) {
    GPL_HIP(hipHostMalloc(reinterpret_cast<void**>(&f.flags), 2 * sizeof(int), hipHostMallocCoherent));
    GPL_HIP(hipEventCreateWithFlags(&f.ev[0], hipEventDisableTiming));
    GPL_HIP(hipEventCreateWithFlags(&f.ev[1], hipEventDisableTiming));
    f.device = dev;
  }
  out = &f;
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

// ---------------------------------------------------------------- entry points

extern "C" size_t gpl_pchol_workspace(const gpl_problem* prob, int k, int prec) {
  if (prob == nullptr || k <= 0 || prob->grid.n <= 0 || prob->grid.ss <= 0) return 0;
  const int npix = prob->grid.n * prob->grid.n, N = npix * prob->grid.ss * prob->grid.ss;
  Sizer s;
  PcBuf b;
  carve_pc(s, npix, N, k, prec, b);
  return s.used;
}

extern "C" int gpl_pchol(const gpl_problem* prob, int k, int prec, double* L, int ldl, double* G, int ldg,
                         int* pivots, double* logdet_P, int* info, void* ws, size_t ws_bytes, hipStream_t stream) {
  Taps taps;
  GPL_TRY(check_pc_problem(prob, taps));
  GPL_REQUIRE(prec == GPL_PREC_FP32 || prec == GPL_PREC_F16X3, "unknown precision %d", prec);
  const int n = prob->grid.n, ss = prob->grid.ss, npix = n * n, N = npix * ss * ss;
  GPL_REQUIRE(k >= kPcBlock && k % kPcBlock == 0, "k=%d must be a positive multiple of %d", k, kPcBlock);
  GPL_REQUIRE(L && G && logdet_P && info, "NULL argument");
  GPL_REQUIRE(ldl >= npix && ldg >= k, "ldl=%d (>= %d) / ldg=%d (>= %d)", ldl, npix, ldg, k);
  GPL_TRY(check_ws(ws, ws_bytes, gpl_pchol_workspace(prob, k, prec)));
  Carver cv(ws, ws_bytes);
  PcBuf b;
  carve_pc(cv, npix, N, k, prec, b);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  rocblas_handle h, h2;
  GPL_TRY(blas_handle(&h, stream, b.blas, kBlasScratch));
  hipStream_t s2;
  hipEvent_t ev[3];  // ev[0], ev[1]: block b of the factor is in (by parity of b); ev[2]: side stream done
  GPL_TRY(side_stream(&s2, ev));
  GPL_TRY(blas_handle(&h2, s2, b.blas2, kBlasScratch, 1));
  MvmCtx mv;
  GPL_TRY(mvm_prepare(mv, prob->kernel.lengthscale, prob->kernel.amplitude, N, prob->px, prob->py, &prob->grid,
                      kPcBlock, prec, b.mvm_ws, b.mvm_bytes, stream));
  const float s2s = (float)kernel_scale2(prob->kernel.lengthscale);
  const double amp2 = prob->kernel.amplitude * prob->kernel.amplitude;
  const double sig2 = prob->noise_sigma * prob->noise_sigma;
  // the side stream starts after everything the caller enqueued so far, and
  // the caller's stream waits for it at the end, error or not
  GPL_HIP(hipEventRecord(ev[1], stream));
  GPL_HIP(hipStreamWaitEvent(s2, ev[1], 0));
  const int rc = [&]() -> int {
    GPL_TRY(border_begin(info, s2));
    hipLaunchKernelGGL(bkb_diag_kernel, dim3(npix), dim3(256), 0, stream, n, ss, taps, s2s, amp2, prob->px, prob->py,
                       b.d);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(dmax_kernel, dim3(1), dim3(1024), 0, stream, npix, b.d, b.dmax);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(zero_ints_kernel, dim3(cdiv(npix, 256)), dim3(256), 0, stream, b.is_piv, npix);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(zero_ints_kernel, dim3(cdiv(mv.plan.nch, 256)), dim3(256), 0, stream, b.chunk_gen,
                       mv.plan.nch);
    GPL_LAUNCH_CHECK();
    const int ldf = round_up(N, 64);
    hipLaunchKernelGGL(set_ints_kernel, dim3(1), dim3(kPcBlock), 0, stream, b.prev, kPcBlock, -1);
    GPL_LAUNCH_CHECK();
    const RhsOut rhs{prec, kPcBlock, mv.bufs.ncp, mv.bufs.Vh, mv.bufs.Vl, mv.bufs.Vp, mv.bufs.inv_scale, nullptr, 0,
                     mv.plan.irank};
    const SpdScratch sw{b.Y, b.W, b.T, b.Dinv, b.ld_part, b.split2, b.split2_elems};
    // on the side stream, once block jb of the factor is in: columns jb .. jb +
    // 63 of G = L^T L (down to row jb + 63), then the bordered inverse of
    // sigma^2 I + G up to that block. The caller's stream records an event
    // after every kSideEvery-th block (a record drains that stream's queue, ~40
    // us), and the side work of the blocks up to it is enqueued after the next
    // block's work on the caller's stream, so that the host keeps that stream
    // fed.
    int pend_lo = 0, pend_hi = 0, pend_g = 0;  // blocks [pend_lo, pend_hi) are in, their side work not enqueued
    auto side_block = [&](int jb) -> int {
      GPL_TRY(split_gemm(h2, rocblas_operation_transpose, rocblas_operation_none, jb + kPcBlock, kPcBlock, npix,
                         kPcSplits, 1.0, L, ldl, L + (size_t)jb * ldl, ldl, 0.0, G + (size_t)jb * ldg, ldg, b.split2,
                         b.split2_elems, s2));
      return border_step(h2, G, ldg, jb, sig2, sw, info, s2);
    };
    auto side_group = [&]() -> int {
      GPL_HIP(hipStreamWaitEvent(s2, ev[pend_g & 1], 0));
      for (; pend_lo < pend_hi; ++pend_lo) GPL_TRY(side_block(pend_lo * kPcBlock));
      return GPL_OK;
    };
    for (int j0 = 0; j0 < k; j0 += kPcBlock) {
      hipLaunchKernelGGL(select_top_kernel, dim3(1), dim3(kSelThreads), 0, stream, npix, b.d, b.cand);
      GPL_LAUNCH_CHECK();
      // columns of B K B^T at the candidates (the matrix-free product)
      // the unit columns are zero outside their footprints: the product skips
      // the chunks that no footprint of this block touches (generation j0 + 1)
      hipLaunchKernelGGL(unit_rhs_kernel, dim3(kPcBlock), dim3(256), 0, stream, n, ss, taps, b.cand, b.prev, rhs,
                         b.chunk_gen, j0 + 1);
      GPL_LAUNCH_CHECK();
      CgGate live;
      live.chunk_gen = b.chunk_gen;
      live.gen = j0 + 1;
      GPL_TRY(mvm_run_prepared(mv, kPcBlock, b.T2, ldf, 0.f, live, stream));
      GPL_TRY(psf_forward_launch(n, ss, taps, kPcBlock, b.T2, ldf, b.Mc, npix, 1.f, 0.f, nullptr, 0, 0.f, nullptr,
                                 0, nullptr, CgGate{}, stream));
      if (j0 == 0) {
        hipLaunchKernelGGL(widen_kernel, dim3(cdiv(npix * kPcBlock, 256)), dim3(256), 0, stream, npix, b.Mc, b.C);
        GPL_LAUNCH_CHECK();
      } else {  // residual columns, by pixel rows: Ct = widened Mc^T - L[cand, :j0] L[:, :j0]^T
        hipLaunchKernelGGL(gather_rows_kernel, dim3(cdiv(kPcBlock * j0, 256)), dim3(256), 0, stream, j0, L, ldl,
                           b.cand, b.Lc);
        GPL_LAUNCH_CHECK();
        GPL_TRY(split_gemm(h, rocblas_operation_none, rocblas_operation_transpose, kPcBlock, npix, j0,
                           std::min(kPcSplits, std::max(1, j0 / 256)), -1.0, b.Lc, kPcBlock, L, ldl, 1.0, b.C,
                           kPcBlock, b.split, b.split_elems, stream, b.Mc));
      }
      hipLaunchKernelGGL(block_pivot_kernel, dim3(1), dim3(64 * kPivWaves), 0, stream, b.C, npix, b.cand, b.dmax,
                         kPcRelTol, b.order, b.taken, b.R);
      GPL_LAUNCH_CHECK();
      double* Lnew = L + (size_t)j0 * ldl;  // = C[:, order] R^{-T}, fixed rows, and the new residual diagonal
      hipLaunchKernelGGL(new_columns_kernel, dim3(cdiv(npix, kNcPix)), dim3(256), 0, stream, npix, b.C, b.order,
                         b.taken, b.R, b.cand, b.d, b.is_piv, Lnew, ldl, pivots, j0);
      GPL_LAUNCH_CHECK();
      // side work of a group whose event was recorded at an earlier block
      if (pend_hi > pend_lo) GPL_TRY(side_group());
      const int blk = j0 / kPcBlock;
      if (blk % kSideEvery == kSideEvery - 1 || j0 + kPcBlock >= k) {
        pend_g = blk / kSideEvery;
        GPL_HIP(hipEventRecord(ev[pend_g & 1], stream));
        pend_hi = blk + 1;
      }
    }
    if (pend_hi > pend_lo) GPL_TRY(side_group());
    GPL_TRY(border_finish(k, sw, b.logdet_g, s2));
    hipLaunchKernelGGL(logdet_p_kernel, dim3(1), dim3(64), 0, s2, npix, k, sig2, b.logdet_g, logdet_P);
    GPL_LAUNCH_CHECK();
    return GPL_OK;
  }();
  GPL_HIP(hipEventRecord(ev[2], s2));
  GPL_HIP(hipStreamWaitEvent(stream, ev[2], 0));
  return rc;
}

extern "C" size_t gpl_pchol_probes_workspace(int npix, int m) {
  if (npix <= 0 || m <= 0) return 0;
  Sizer s;
  s.take<double>((size_t)npix * m);
  s.take<char>(kBlasScratch);
  return s.used;
}

extern "C" int gpl_pchol_probes(int npix, int k, const double* L, int ldl, double noise_sigma, int m, const double* g,
                                int ldg, const float* hn, int ldh, float* Z, int ldz, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
  GPL_REQUIRE(npix >= 1 && k >= 1 && m >= 0, "bad sizes");
  if (m == 0) return GPL_OK;
  GPL_REQUIRE(L && g && hn && Z, "NULL argument");
  GPL_REQUIRE(ldl >= npix && ldg >= k && ldh >= npix && ldz >= npix, "leading dimension too small");
  GPL_REQUIRE(noise_sigma > 0 && std::isfinite(noise_sigma), "noise_sigma must be > 0");
  GPL_TRY(check_ws(ws, ws_bytes, gpl_pchol_probes_workspace(npix, m)));
  Carver cv(ws, ws_bytes);
  double* Lg = cv.take<double>((size_t)npix * m);
  void* scratch = cv.take<char>(kBlasScratch);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  rocblas_handle h;
  GPL_TRY(blas_handle(&h, stream, scratch, kBlasScratch));
  const double one = 1.0, zero = 0.0;
  if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, npix, m, k, &one, L, ldl, g, ldg, &zero, Lg,
                    npix) != rocblas_status_success) {
    set_error("rocblas_dgemm (probes) failed");
    return GPL_EHIP;
  }
  hipLaunchKernelGGL(probe_finish_kernel, dim3(cdiv(npix, 256), m), dim3(256), 0, stream, npix, Lg, noise_sigma, hn,
                     ldh, Z, ldz);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" size_t gpl_pcg_solve_workspace(const gpl_problem* prob, int k, int nrhs, int prec) {
  if (prob == nullptr || nrhs <= 0 || prob->grid.n <= 0 || prob->grid.ss <= 0) return 0;
  const int n = prob->grid.n, ss = prob->grid.ss, npix = n * n, N = npix * ss * ss;
  Sizer s;
  PcgBuf b;
  carve_pcg(s, npix, N, n, ss, k, nrhs, prec, b);
  return s.used;
}

extern "C" int gpl_pcg_solve(const gpl_problem* prob, int k, const double* L, int ldl, const double* G, int ldg,
                             int nrhs, const float* Bm, int ldb, float* X, int ldx, double tol, int max_iter,
                             int fixed_iters, int n_lanczos, double* lanczos_ab, double* rz0, int* iters,
                             double* relres, double* true_relres, int* status, int prec, int check_every, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  Taps taps;
  GPL_TRY(check_pc_problem(prob, taps));
  GPL_REQUIRE(prec == GPL_PREC_FP32 || prec == GPL_PREC_F16X3, "unknown precision %d", prec);
  GPL_REQUIRE(nrhs >= 1 && nrhs <= 65535, "nrhs=%d out of range", nrhs);
  const int n = prob->grid.n, ss = prob->grid.ss, npix = n * n, N = npix * ss * ss;
  GPL_REQUIRE(k >= 1 && L && G && ldl >= npix && ldg >= k, "bad preconditioner arguments");
  GPL_REQUIRE(Bm && X && ldb >= npix && ldx >= npix, "bad right-hand side or solution arguments");
  GPL_REQUIRE(tol >= 0 && max_iter >= 0 && fixed_iters >= 0 && n_lanczos >= 0 && check_every >= 0,
              "negative tol/iteration counts");
  GPL_REQUIRE(n_lanczos == 0 || lanczos_ab != nullptr, "lanczos_ab is NULL");
  GPL_TRY(check_ws(ws, ws_bytes, gpl_pcg_solve_workspace(prob, k, nrhs, prec)));
  Carver cv(ws, ws_bytes);
  PcgBuf b;
  carve_pcg(cv, npix, N, n, ss, k, nrhs, prec, b);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  rocblas_handle h;
  GPL_TRY(blas_handle(&h, stream, b.blas, kBlasScratch));
  PollFlags* poll = nullptr;
  if (check_every > 0) GPL_TRY(pcg_poll(poll));
  MvmCtx mv;
  GPL_TRY(mvm_prepare(mv, prob->kernel.lengthscale, prob->kernel.amplitude, N, prob->px, prob->py, &prob->grid, nrhs,
                      prec, b.mvm_ws, b.mvm_bytes, stream));
  const RhsOut rhs_out{prec, nrhs, mv.bufs.ncp, mv.bufs.Vh, mv.bufs.Vl, mv.bufs.Vp, mv.bufs.inv_scale, b.pmax, b.nb,
                       mv.plan.irank};
  const float sigma2 = (float)(prob->noise_sigma * prob->noise_sigma);
  const double inv_s = 1.0 / (prob->noise_sigma * prob->noise_sigma);
  const int nb = b.nb;
  const dim3 gv(nb, nrhs);
  const int limit = fixed_iters > 0 ? fixed_iters : max_iter;

  // R = b, Z = P^{-1} b, P = Z, states
  hipLaunchKernelGGL(pcg_init_kernel, gv, dim3(256), 0, stream, npix, Bm, ldb, X, ldx, b.R, b.ldv, b.rr_part, nb);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(pcg_widen_kernel, gv, dim3(256), 0, stream, npix, b.R, b.ldv, b.R64, b.Z64);
  GPL_LAUNCH_CHECK();
  GPL_TRY(woodbury(h, npix, k, L, ldl, G, ldg, nrhs, b.R64, b.Z64, b.ldv, b.W, b.W2, b.split, b.split_elems, stream));
  hipLaunchKernelGGL(pcg_zfinish_kernel, gv, dim3(256), 0, stream, npix, b.Z64, b.ldv, inv_s, b.R, b.Z, b.rz_part,
                     nb, (const PcgState*)nullptr, (const int*)nullptr);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(pcg_init_p_kernel, gv, dim3(256), 0, stream, npix, b.Z, b.P, b.ldv, b.pmax, nb);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(pcg_init_state_kernel, dim3(1), dim3(256), 0, stream, nrhs, b.rr_part, b.rz_part, nb, b.st[0],
                     b.st[1], b.bb, rz0, b.n_active, limit);
  GPL_LAUNCH_CHECK();

  const int chunk = check_every > 0 ? check_every : std::max(limit, 1);
  const int nchunks = cdiv(limit, chunk);
  int last_end = 0;
  auto enqueue_chunk = [&](int kc) -> int {
    const int end = std::min(limit, (kc + 1) * chunk);
    for (int it = kc * chunk; it < end; ++it) {
      const int p = it & 1;
      CgGate gate;
      gate.n_active = b.n_active + p;
      GPL_TRY(psf_adjoint_rhs_launch(n, ss, taps, nrhs, b.P, b.ldv, rhs_out, gate, stream));
      GPL_TRY(mvm_run_prepared(mv, nrhs, b.T2, b.ldf, 0.f, gate, stream));
      GPL_TRY(psf_forward_launch(n, ss, taps, nrhs, b.T2, b.ldf, b.AP, b.ldv, 1.f, 0.f, b.P, b.ldv, sigma2, b.P,
                                 b.ldv, b.pap_part, gate, stream));
      hipLaunchKernelGGL(pcg_update1_kernel, gv, dim3(256), 0, stream, npix, X, ldx, b.R, b.P, b.AP, b.ldv, b.R64,
                         b.Z64, b.pap_part, b.ntiles, b.rr_part, nb, b.st[p], b.st[1 - p], b.n_active + p,
                         b.n_active + (1 - p));
      GPL_LAUNCH_CHECK();
      GPL_TRY(woodbury(h, npix, k, L, ldl, G, ldg, nrhs, b.R64, b.Z64, b.ldv, b.W, b.W2, b.split, b.split_elems, stream));
      hipLaunchKernelGGL(pcg_zfinish_kernel, gv, dim3(256), 0, stream, npix, b.Z64, b.ldv, inv_s, b.R, b.Z,
                         b.rz_part, nb, (const PcgState*)b.st[p], (const int*)(b.n_active + p));
      GPL_LAUNCH_CHECK();
      hipLaunchKernelGGL(pcg_update2_kernel, gv, dim3(256), 0, stream, npix, b.Z, b.P, b.ldv, b.rr_part, b.rz_part,
                         nb, b.st[p], b.st[1 - p], b.bb, b.n_active + p, b.n_active + (1 - p), tol, max_iter,
                         fixed_iters, n_lanczos, lanczos_ab, b.pmax);
      GPL_LAUNCH_CHECK();
    }
    last_end = end;
    if (!poll) return GPL_OK;
    hipLaunchKernelGGL(pcg_snapshot_kernel, dim3(1), dim3(64), 0, stream, b.n_active + (end & 1),
                       poll->flags + (kc & 1));
    GPL_LAUNCH_CHECK();
    GPL_HIP(hipEventRecord(poll->ev[kc & 1], stream));
    return GPL_OK;
  };
  if (nchunks > 0 && !poll) {
    GPL_TRY(enqueue_chunk(0));
  } else if (nchunks > 0) {
    GPL_TRY(enqueue_chunk(0));
    for (int kc = 0; kc < nchunks; ++kc) {
      if (kc + 1 < nchunks) GPL_TRY(enqueue_chunk(kc + 1));
      GPL_HIP(hipEventSynchronize(poll->ev[kc & 1]));
      if (poll->flags[kc & 1] == 0) break;
    }
  }
  const int fp = last_end & 1;
  hipLaunchKernelGGL(pcg_finalize_kernel, dim3(cdiv(nrhs, 256)), dim3(256), 0, stream, nrhs, b.st[fp], b.bb, iters,
                     relres, status, n_lanczos, lanczos_ab);
  GPL_LAUNCH_CHECK();
  if (true_relres) {
    hipLaunchKernelGGL(pcg_absmax_kernel, gv, dim3(256), 0, stream, npix, X, ldx, b.pmax, nb);
    GPL_LAUNCH_CHECK();
    GPL_TRY(psf_adjoint_rhs_launch(n, ss, taps, nrhs, X, ldx, rhs_out, CgGate{}, stream));
    GPL_TRY(mvm_run_prepared(mv, nrhs, b.T2, b.ldf, 0.f, CgGate{}, stream));
    GPL_TRY(psf_forward_launch(n, ss, taps, nrhs, b.T2, b.ldf, b.AP, b.ldv, 1.f, 0.f, X, ldx, sigma2, nullptr, 0,
                               nullptr, CgGate{}, stream));
    hipLaunchKernelGGL(pcg_true_residual_kernel, gv, dim3(256), 0, stream, npix, Bm, ldb, b.AP, b.ldv, b.rr_part, nb);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(pcg_true_residual_fold_kernel, dim3(cdiv(nrhs, 256)), dim3(256), 0, stream, nrhs, b.rr_part,
                       nb, b.bb, true_relres);
    GPL_LAUNCH_CHECK();
  }
  return GPL_OK;
}
