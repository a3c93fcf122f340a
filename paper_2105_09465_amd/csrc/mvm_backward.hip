// Adjoint of the kernel-matrix product with kernel tiles recomputed (the paper
// differentiates its matrix-free product automatically, Sec. 3.3; here the
// adjoint is written out). For F = sum_c w_c a_c^T K b_c with
// K_ij = a^2 exp(-|p_i - p_j|^2 / (2 l^2)) (eq. "grbf"):
//   s_ij     = sum_c w_c (a_ic b_jc + a_jc b_ic)
//   dF/dp_i  = -(1/l^2) sum_j K_ij s_ij (p_i - p_j)
//   dF/dl    = (1/2) sum_ij K_ij s_ij |p_i - p_j|^2 / l^3
//   dF/da    = sum_ij K_ij s_ij / a          (= 2F/a)
// The points are taken in the order of the product's tile plan (a Hilbert
// sort), so that runs of consecutive points are compact. Source chunks (32
// points) whose box gap g to a row block's box gives s2 g^2 >= kSkipBackward
// are skipped: every kernel value there is at most a^2 2^-36, so each skipped
// term K s (p_i - p_j) is below 2^-36 of the same term at kernel value a^2 (the
// precision form's product treats these values as zero as well).
// Each lane owns R rows i and keeps w_c a_ic, w_c b_ic in registers; source
// tiles of 256 points with their a_j, b_j are staged in LDS. The source range is
// split across workgroups; per-slice position gradients and per-block FP64
// hyperparameter sums are reduced in a fixed order by later kernels.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"
#include "tileplan.hpp"

namespace gpl {

constexpr int kBJ = 256;              // points per source tile (8 chunks of the plan)
constexpr int kMaxPass = 16;          // column pairs per pass
constexpr float kSkipBackward = kSkipF16x3;
static_assert(kBJ % kChunk == 0, "source tiles are whole chunks");

struct WChunk {
  float w[kMaxPass];  // weights of the (up to 16) column pairs of one pass
};

struct BwdPlan {
  int R, rows, nrb, S, jlen, ldg, nchunk;
};

static BwdPlan bwd_plan(int n, int npairs) {
  BwdPlan p;
  p.R = n >= 16384 ? 2 : 1;
  p.rows = 256 * p.R;
  p.nrb = cdiv(n, p.rows);
  // about 2048 workgroups: after the cut their work varies, and many short
  // workgroups keep the compute units filled
  const int target = 2048;
  const int S = std::max(1, std::min(target / p.nrb, cdiv(n, kBJ)));
  p.jlen = round_up(cdiv(n, S), kBJ);
  p.S = cdiv(n, p.jlen);
  p.ldg = round_up(n, 64);
  p.nchunk = 0;
  for (int c0 = 0; c0 < npairs;) {
    const int left = npairs - c0;
    c0 += left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    ++p.nchunk;
  }
  return p;
}

// Box of the sorted points [kBJ t, kBJ t + kBJ): the union of the plan's chunk
// boxes (empty past the last chunk).
__device__ __forceinline__ float4 source_tile_box(const float4* __restrict__ cbox, int nch, int t) {
  float4 b = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
#pragma unroll
  for (int k = 0; k < kBJ / kChunk; ++k) {
    const int c = t * (kBJ / kChunk) + k;
    if (c < nch) {
      const float4 q = cbox[c];
      b = make_float4(fminf(b.x, q.x), fmaxf(b.y, q.y), fminf(b.z, q.z), fmaxf(b.w, q.w));
    }
  }
  return b;
}

// Bit k set when chunk kBJ/kChunk t + k of source tile t is within the cutoff of
// the row box rb (the same value in every thread of a workgroup).
__device__ __forceinline__ unsigned source_chunks_live(const float4* __restrict__ cbox, int nch, int t,
                                                       const float4& rb, float s2) {
  unsigned m = 0u;
#pragma unroll
  for (int k = 0; k < kBJ / kChunk; ++k) {
    const int c = t * (kBJ / kChunk) + k;
    if (c < nch && boxes_live(rb, cbox[c], s2, kSkipBackward)) m |= 1u << k;
  }
  return m;
}

// Columns c0 .. c0 + nc of A and Bv in the plan's order: As[c][j] = A[c0 + c][perm[j]].
__global__ void bwd_gather_kernel(int n, int nc, int c0, const int* __restrict__ perm, const float* __restrict__ A,
                                  int lda, const float* __restrict__ Bv, int ldb, float* __restrict__ As,
                                  float* __restrict__ Bs, int ldp) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int i = perm[j];
  for (int c = 0; c < nc; ++c) {
    As[(size_t)c * ldp + j] = A[(size_t)(c0 + c) * lda + i];
    Bs[(size_t)c * ldp + j] = Bv[(size_t)(c0 + c) * ldb + i];
  }
}

// part_g[slice][2][ldg]: position-gradient partials of the sorted rows;
// part_h[slice][block][2]: FP64 sums of K s d^2 and K s.
template <int NC, int R>
__global__ __launch_bounds__(256) void mvm_bwd_kernel(int n, const float* __restrict__ xs,
                                                      const float* __restrict__ ys, const float4* __restrict__ cbox,
                                                      int nch, float s2, float amp2, const float* __restrict__ As,
                                                      const float* __restrict__ Bs, int ldp, WChunk w, int jlen,
                                                      double* __restrict__ part_g, int ldg,
                                                      double* __restrict__ part_h) {
  __shared__ float sx[kBJ], sy[kBJ];
  __shared__ __attribute__((aligned(16))) float sa[kBJ * NC];
  __shared__ __attribute__((aligned(16))) float sb[kBJ * NC];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * (256 * R);
  const int jbeg = blockIdx.y * jlen;
  const int jend = min(n, jbeg + jlen);
  // the row block's box (the same value in every thread, so the tile test below
  // takes the same branch in the whole workgroup)
  float4 rb = source_tile_box(cbox, nch, row0 / kBJ);
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const float4 q = source_tile_box(cbox, nch, row0 / kBJ + r);
    rb = make_float4(fminf(rb.x, q.x), fmaxf(rb.y, q.y), fminf(rb.z, q.z), fmaxf(rb.w, q.w));
  }
  // this wave's rows: the 64-point row tiles row0/64 + w + 4r (r < R); their box
  // (the same value in every lane) selects the chunks the wave computes
  const int wv = tid >> 6;
  float4 wb4 = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int k = 0; k < kChunksPerTile; ++k) {
      const int c = (row0 / kRowTile + wv + 4 * r) * kChunksPerTile + k;
      if (c < nch) {
        const float4 q = cbox[c];
        wb4 = make_float4(fminf(wb4.x, q.x), fmaxf(wb4.y, q.y), fminf(wb4.z, q.z), fmaxf(wb4.w, q.w));
      }
    }
  }
  float xi[R], yi[R], wa[R][NC], wb[R][NC];
  double gx[R], gy[R];       // FP64 accumulation: the gradient terms partly cancel
  double hl = 0.0, hf = 0.0;  // per-lane sums of K s d^2 and K s
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = row0 + r * 256 + tid;
    const bool ok = i < n;
    xi[r] = ok ? xs[i] : 0.f;
    yi[r] = ok ? ys[i] : 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      wa[r][c] = ok ? w.w[c] * As[(size_t)c * ldp + i] : 0.f;
      wb[r][c] = ok ? w.w[c] * Bs[(size_t)c * ldp + i] : 0.f;
    }
    gx[r] = 0.0;
    gy[r] = 0.0;
  }
  for (int jt = jbeg; jt < jend; jt += kBJ) {
    const unsigned live = source_chunks_live(cbox, nch, jt / kBJ, rb, s2);
    if (live == 0u) continue;
    __syncthreads();
    const int j = jt + tid;
    const bool ok = j < jend;
    sx[tid] = ok ? xs[j] : 0.f;
    sy[tid] = ok ? ys[j] : 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      sa[tid * NC + c] = ok ? As[(size_t)c * ldp + j] : 0.f;
      sb[tid * NC + c] = ok ? Bs[(size_t)c * ldp + j] : 0.f;
    }
    __syncthreads();
    const unsigned wlive = source_chunks_live(cbox, nch, jt / kBJ, wb4, s2);  // a subset of live
    for (int g = 0; g < kBJ / kChunk; ++g) {
      if (!((wlive >> g) & 1u)) continue;
#pragma unroll 2
    for (int t = g * kChunk; t < (g + 1) * kChunk; ++t) {
      const float xj = sx[t], yj = sy[t];
      float aj[NC], bj[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        aj[c] = sa[t * NC + c];
        bj[c] = sb[t * NC + c];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < NC; ++c) s = fmaf(wa[r][c], bj[c], fmaf(wb[r][c], aj[c], s));
        const float dx = xi[r] - xj, dy = yi[r] - yj;
        const float d2 = fmaf(dx, dx, dy * dy);
        const double kt = (double)(amp2 * exp2_fast(-(d2 * s2)) * s);
        gx[r] = fma(kt, (double)dx, gx[r]);
        gy[r] = fma(kt, (double)dy, gy[r]);
        hl = fma(kt, (double)d2, hl);
        hf += kt;
      }
    }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = row0 + r * 256 + tid;
    if (i < n) {
      part_g[((size_t)blockIdx.y * 2 + 0) * ldg + i] = gx[r];
      part_g[((size_t)blockIdx.y * 2 + 1) * ldg + i] = gy[r];  // slice partials kept in FP64
    }
  }
  const size_t hb = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
  const double sl = block_sum_double(hl, red);
  if (tid == 0) part_h[hb + 0] = sl;
  const double sf = block_sum_double(hf, red);
  if (tid == 0) part_h[hb + 1] = sf;
}

// gacc[k][i] (+)= sum over the slices of one pass of part_g[slice][k][i], in slice order.
__global__ void bwd_reduce_pos_kernel(int n, int nslices, const double* __restrict__ part_g, int ldg, int first,
                                      double* __restrict__ gacc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sx = first ? 0.0 : gacc[i], sy = first ? 0.0 : gacc[ldg + i];
  for (int k = 0; k < nslices; ++k) {
    sx += part_g[((size_t)k * 2 + 0) * ldg + i];
    sy += part_g[((size_t)k * 2 + 1) * ldg + i];
  }
  gacc[i] = sx;
  gacc[ldg + i] = sy;
}

// gpx[perm[i]] += -(1/l^2) gacc[0][i]; same for y.
__global__ void bwd_store_pos_kernel(int n, const int* __restrict__ perm, const double* __restrict__ gacc, int ldg,
                                     double inv_l2, float* gpx, float* gpy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int dst = perm[i];
  gpx[dst] += (float)(-inv_l2 * gacc[i]);
  gpy[dst] += (float)(-inv_l2 * gacc[ldg + i]);
}

// g_hyp[0] = (1/2) sum K s d^2 / l^3, g_hyp[1] = sum K s / a (one workgroup of
// 256 threads, each summing a fixed stride of the blocks, then a fixed tree).
__global__ __launch_bounds__(256) void bwd_reduce_hyp_kernel(int nblocks_total, const double* part_h, double l,
                                                             double a, double* g_hyp) {
  __shared__ double red[4];
  double sl = 0.0, sf = 0.0;
  for (int b = threadIdx.x; b < nblocks_total; b += blockDim.x) {
    sl += part_h[2 * b + 0];
    sf += part_h[2 * b + 1];
  }
  sl = block_sum_double(sl, red);
  sf = block_sum_double(sf, red);
  if (threadIdx.x == 0) {
    g_hyp[0] = 0.5 * sl / (l * l * l);
    g_hyp[1] = sf / a;
  }
}

struct BwdBufs {
  TilePlan plan;
  float *As, *Bs;  // [kMaxPass][ldg] columns of one pass in the plan's order
  double *part_g, *gacc, *part_h;
};

template <class Cv>
static void carve_bwd(Cv& cv, int n, const BwdPlan& p, BwdBufs& b) {
  plan_carve(cv, n, b.plan);
  b.As = cv.template take<float>((size_t)kMaxPass * p.ldg);
  b.Bs = cv.template take<float>((size_t)kMaxPass * p.ldg);
  b.part_g = cv.template take<double>((size_t)p.S * 2 * p.ldg);
  b.gacc = cv.template take<double>((size_t)2 * p.ldg);
  b.part_h = cv.template take<double>((size_t)p.nchunk * p.S * p.nrb * 2);
}

template <int NC>
static void launch_bwd(const BwdPlan& p, int n, const TilePlan& P, float s2, float amp2, const float* As,
                       const float* Bs, const WChunk& w, double* part_g, double* part_h, hipStream_t stream) {
  dim3 grid(p.nrb, p.S);
  if (p.R == 2)
    hipLaunchKernelGGL((mvm_bwd_kernel<NC, 2>), grid, dim3(256), 0, stream, n, P.xs, P.ys, P.cbox, P.nch, s2, amp2,
                       As, Bs, p.ldg, w, p.jlen, part_g, p.ldg, part_h);
  else
    hipLaunchKernelGGL((mvm_bwd_kernel<NC, 1>), grid, dim3(256), 0, stream, n, P.xs, P.ys, P.cbox, P.nch, s2, amp2,
                       As, Bs, p.ldg, w, p.jlen, part_g, p.ldg, part_h);
}

}  // namespace gpl

using namespace gpl;

extern "C" size_t gpl_gp_kernel_mvm_backward_workspace(int n, int npairs) {
  if (n <= 0 || npairs <= 0) return 0;
  const BwdPlan p = bwd_plan(n, npairs);
  Sizer s;
  BwdBufs b;
  carve_bwd(s, n, p, b);
  return s.used;
}

extern "C" int gpl_gp_kernel_mvm_backward(const gpl_kernel* kern, int n, const float* px, const float* py,
                                          int npairs, const float* A, int lda, const float* Bv, int ldb,
                                          const double* w, float* gpx, float* gpy, double* g_hyp, void* ws,
                                          size_t ws_bytes, hipStream_t stream) {
  GPL_TRY(check_kernel(kern));
  GPL_REQUIRE(n >= 1 && npairs >= 1 && npairs <= 4096, "n=%d npairs=%d out of range", n, npairs);
  GPL_REQUIRE(px && py && A && Bv && w && gpx && gpy && g_hyp, "NULL argument");
  GPL_REQUIRE(lda >= n && ldb >= n, "lda/ldb must be >= n");
  GPL_REQUIRE(kern->amplitude != 0.0, "amplitude must be non-zero for the amplitude gradient");
  for (int c = 0; c < npairs; ++c) GPL_REQUIRE(std::isfinite(w[c]), "weight %d is not finite", c);
  GPL_TRY(check_ws(ws, ws_bytes, gpl_gp_kernel_mvm_backward_workspace(n, npairs)));
  const BwdPlan p = bwd_plan(n, npairs);
  Carver cv(ws, ws_bytes);
  BwdBufs b;
  carve_bwd(cv, n, p, b);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  const float s2 = (float)kernel_scale2(kern->lengthscale);
  const float amp2 = (float)(kern->amplitude * kern->amplitude);
  GPL_TRY(plan_build(b.plan, n, px, py, nullptr, s2, kSkipFp32Exact, kSkipFp32Exact, stream));
  int chunk = 0;
  for (int c0 = 0; c0 < npairs; ++chunk) {
    const int left = npairs - c0;
    const int nc = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    WChunk wd;
    for (int c = 0; c < kMaxPass; ++c) wd.w[c] = c < nc ? (float)w[c0 + c] : 0.f;
    hipLaunchKernelGGL(bwd_gather_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, nc, c0, b.plan.perm, A, lda,
                       Bv, ldb, b.As, b.Bs, p.ldg);
    GPL_LAUNCH_CHECK();
    double* ph = b.part_h + (size_t)chunk * p.S * p.nrb * 2;
    switch (nc) {
      case 16: launch_bwd<16>(p, n, b.plan, s2, amp2, b.As, b.Bs, wd, b.part_g, ph, stream); break;
      case 8: launch_bwd<8>(p, n, b.plan, s2, amp2, b.As, b.Bs, wd, b.part_g, ph, stream); break;
      case 4: launch_bwd<4>(p, n, b.plan, s2, amp2, b.As, b.Bs, wd, b.part_g, ph, stream); break;
      case 2: launch_bwd<2>(p, n, b.plan, s2, amp2, b.As, b.Bs, wd, b.part_g, ph, stream); break;
      default: launch_bwd<1>(p, n, b.plan, s2, amp2, b.As, b.Bs, wd, b.part_g, ph, stream); break;
    }
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(bwd_reduce_pos_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, p.S, b.part_g, p.ldg,
                       chunk == 0 ? 1 : 0, b.gacc);
    GPL_LAUNCH_CHECK();
    c0 += nc;
  }
  const double inv_l2 = 1.0 / (kern->lengthscale * kern->lengthscale);
  hipLaunchKernelGGL(bwd_store_pos_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, b.plan.perm, b.gacc, p.ldg,
                     inv_l2, gpx, gpy);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(bwd_reduce_hyp_kernel, dim3(1), dim3(256), 0, stream, p.nchunk * p.S * p.nrb, b.part_h,
                     kern->lengthscale, kern->amplitude, g_hyp);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
