// Adjoint of the kernel-matrix product with kernel tiles recomputed (the paper
// differentiates its matrix-free product automatically, Sec. 3.3; here the
// adjoint is written out). For F = sum_c w_c a_c^T K b_c with
// K_ij = a^2 exp(-|p_i - p_j|^2 / (2 l^2)) (eq. "grbf"):
//   s_ij     = sum_c w_c (a_ic b_jc + a_jc b_ic)
//   dF/dp_i  = -(1/l^2) sum_j K_ij s_ij (p_i - p_j)
//   dF/dl    = (1/2) sum_ij K_ij s_ij |p_i - p_j|^2 / l^3
//   dF/da    = sum_ij K_ij s_ij / a          (= 2F/a)
// Each lane owns R rows i and keeps w_c a_ic, w_c b_ic in registers; tiles of
// 256 source points with their a_j, b_j are staged in LDS. The source range is
// split across workgroups; per-slice position gradients and per-block FP64
// hyperparameter sums are reduced in a fixed order by a second kernel.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace gpl {

constexpr int kBJ = 256;

struct WChunk {
  float w[16];  // weights of the (up to 16) column pairs of one pass
};

struct BwdPlan {
  int R, rows, nrb, S, jlen, ldg, nchunk;
};

static BwdPlan bwd_plan(int n, int npairs) {
  BwdPlan p;
  p.R = n >= 16384 ? 2 : 1;
  p.rows = 256 * p.R;
  p.nrb = cdiv(n, p.rows);
  const int target = 1024;
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

// part_g[chunk][slice][2][ldg]: position-gradient partials; part_h[chunk][slice][block][2]: FP64 sums of
// K s d^2 and K s.
template <int NC, int R>
__global__ __launch_bounds__(256) void mvm_bwd_kernel(int n, const float* __restrict__ px,
                                                      const float* __restrict__ py, float s2, float amp2,
                                                      const float* __restrict__ A, int lda,
                                                      const float* __restrict__ Bv, int ldb, WChunk w,
                                                      int c0, int jlen, double* __restrict__ part_g, int ldg,
                                                      double* __restrict__ part_h) {
  __shared__ float sx[kBJ], sy[kBJ];
  __shared__ __attribute__((aligned(16))) float sa[kBJ * NC];
  __shared__ __attribute__((aligned(16))) float sb[kBJ * NC];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * (256 * R);
  const int jbeg = blockIdx.y * jlen;
  const int jend = min(n, jbeg + jlen);
  float xi[R], yi[R], wa[R][NC], wb[R][NC];
  double gx[R], gy[R];       // FP64 accumulation: the gradient terms partly cancel
  double hl = 0.0, hf = 0.0;  // per-lane sums of K s d^2 and K s
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = row0 + r * 256 + tid;
    const bool ok = i < n;
    xi[r] = ok ? px[i] : 0.f;
    yi[r] = ok ? py[i] : 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      wa[r][c] = ok ? w.w[c] * A[(size_t)(c0 + c) * lda + i] : 0.f;
      wb[r][c] = ok ? w.w[c] * Bv[(size_t)(c0 + c) * ldb + i] : 0.f;
    }
    gx[r] = 0.0;
    gy[r] = 0.0;
  }
  for (int jt = jbeg; jt < jend; jt += kBJ) {
    __syncthreads();
    const int j = jt + tid;
    const bool ok = j < jend;
    sx[tid] = ok ? px[j] : 0.f;
    sy[tid] = ok ? py[j] : 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      sa[tid * NC + c] = ok ? A[(size_t)(c0 + c) * lda + j] : 0.f;
      sb[tid * NC + c] = ok ? Bv[(size_t)(c0 + c) * ldb + j] : 0.f;
    }
    __syncthreads();
#pragma unroll 2
    for (int t = 0; t < kBJ; ++t) {
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

// gpx[i] += -(1/l^2) sum_{chunk, slice} gx; same for y.
__global__ void bwd_reduce_pos_kernel(int n, int nslices_total, const double* __restrict__ part_g, int ldg,
                                      double inv_l2, float* gpx, float* gpy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sx = 0.0, sy = 0.0;
  for (int k = 0; k < nslices_total; ++k) {
    sx += part_g[((size_t)k * 2 + 0) * ldg + i];
    sy += part_g[((size_t)k * 2 + 1) * ldg + i];
  }
  gpx[i] += (float)(-inv_l2 * sx);
  gpy[i] += (float)(-inv_l2 * sy);
}

// g_hyp[0] = (1/2) sum K s d^2 / l^3, g_hyp[1] = sum K s / a.
__global__ void bwd_reduce_hyp_kernel(int nblocks_total, const double* part_h, double l, double a, double* g_hyp) {
  if (threadIdx.x != 0) return;
  double sl = 0.0, sf = 0.0;
  for (int b = 0; b < nblocks_total; ++b) {
    sl += part_h[2 * b + 0];
    sf += part_h[2 * b + 1];
  }
  g_hyp[0] = 0.5 * sl / (l * l * l);
  g_hyp[1] = sf / a;
}

template <class Cv>
static void carve_bwd(Cv& cv, const BwdPlan& p, double** part_g, double** part_h) {
  *part_g = cv.template take<double>((size_t)p.nchunk * p.S * 2 * p.ldg);
  *part_h = cv.template take<double>((size_t)p.nchunk * p.S * p.nrb * 2);
}

template <int NC>
static void launch_bwd(const BwdPlan& p, int n, const float* px, const float* py, float s2, float amp2, const float* A,
                       int lda, const float* Bv, int ldb, const WChunk& w, int c0, double* part_g, double* part_h,
                       hipStream_t stream) {
  dim3 grid(p.nrb, p.S);
  if (p.R == 2)
    hipLaunchKernelGGL((mvm_bwd_kernel<NC, 2>), grid, dim3(256), 0, stream, n, px, py, s2, amp2, A, lda, Bv, ldb, w,
                       c0, p.jlen, part_g, p.ldg, part_h);
  else
    hipLaunchKernelGGL((mvm_bwd_kernel<NC, 1>), grid, dim3(256), 0, stream, n, px, py, s2, amp2, A, lda, Bv, ldb, w,
                       c0, p.jlen, part_g, p.ldg, part_h);
}

}  // namespace gpl

using namespace gpl;

extern "C" size_t gpl_gp_kernel_mvm_backward_workspace(int n, int npairs) {
  if (n <= 0 || npairs <= 0) return 0;
  const BwdPlan p = bwd_plan(n, npairs);
  Sizer s;
  double *b, *c;
  carve_bwd(s, p, &b, &c);
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
  double *part_g, *part_h;
  carve_bwd(cv, p, &part_g, &part_h);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  const float s2 = (float)kernel_scale2(kern->lengthscale);
  const float amp2 = (float)(kern->amplitude * kern->amplitude);
  int chunk = 0;
  for (int c0 = 0; c0 < npairs; ++chunk) {
    const int left = npairs - c0;
    const int nc = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    WChunk wd;
    for (int c = 0; c < 16; ++c) wd.w[c] = c < nc ? (float)w[c0 + c] : 0.f;
    double* pg = part_g + (size_t)chunk * p.S * 2 * p.ldg;
    double* ph = part_h + (size_t)chunk * p.S * p.nrb * 2;
    switch (nc) {
      case 16: launch_bwd<16>(p, n, px, py, s2, amp2, A, lda, Bv, ldb, wd, c0, pg, ph, stream); break;
      case 8: launch_bwd<8>(p, n, px, py, s2, amp2, A, lda, Bv, ldb, wd, c0, pg, ph, stream); break;
      case 4: launch_bwd<4>(p, n, px, py, s2, amp2, A, lda, Bv, ldb, wd, c0, pg, ph, stream); break;
      case 2: launch_bwd<2>(p, n, px, py, s2, amp2, A, lda, Bv, ldb, wd, c0, pg, ph, stream); break;
      default: launch_bwd<1>(p, n, px, py, s2, amp2, A, lda, Bv, ldb, wd, c0, pg, ph, stream); break;
    }
    GPL_LAUNCH_CHECK();
    c0 += nc;
  }
  const double inv_l2 = 1.0 / (kern->lengthscale * kern->lengthscale);
  hipLaunchKernelGGL(bwd_reduce_pos_kernel, dim3(cdiv(n, 256)), dim3(256), 0, stream, n, p.nchunk * p.S, part_g,
                     p.ldg, inv_l2, gpx, gpy);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(bwd_reduce_hyp_kernel, dim3(1), dim3(64), 0, stream, p.nchunk * p.S * p.nrb, part_h,
                     kern->lengthscale, kern->amplitude, g_hyp);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}
