// Matrix-free kernel-matrix product Y = K V + beta Y with the RBF kernel of
// Sec. 3.1 (eq. "grbf"), K_ij = a^2 exp(-|p_i - p_j|^2 / (2 l^2)). The paper
// forms this product on the fly, never storing K (Sec. 3.3, transmission
// matrix "too large to store"); here the same holds on gfx950.
//
// FP32 VALU form (this file): each workgroup owns 256*R output rows (R rows per
// lane, coalesced SoA loads) and one slice of the source points. Source points
// and the matching rows of V are staged in LDS in tiles of 256; every lane
// forms its exp tile in registers from exact coordinate differences
// (d = p_i - p_j first, then the 1/(2 l^2) scale, so no cancellation error
// enters from large absolute coordinates) and accumulates NC right-hand sides
// with FMAs. Slices of the source points give enough workgroups to fill all
// CUs; their partial products are summed in a fixed order by a second kernel,
// so results are bitwise reproducible.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"
#include "mvm_mfma.hpp"
#include "timing.hpp"

namespace gpl {

constexpr int kTJ = 256;
constexpr int kFp32MfmaMinCols = 4;

struct MvmPlan {
  int R;        // rows per lane
  int rows;     // rows per workgroup
  int nrb;      // row blocks
  int S;        // source-point slices
  int jlen;     // points per slice (multiple of kTJ)
  int ldp;      // leading dimension of the partial buffer
};

static MvmPlan valu_plan(int n) {
  MvmPlan p;
  p.R = n >= 16384 ? 4 : 1;
  p.rows = 256 * p.R;
  p.nrb = cdiv(n, p.rows);
  const int target = 1024;  // workgroups: 4 per CU
  int S = std::max(1, std::min(target / p.nrb, cdiv(n, kTJ)));
  p.jlen = round_up(cdiv(n, S), kTJ);
  p.S = cdiv(n, p.jlen);
  p.ldp = round_up(n, 64);
  return p;
}

template <int NC, int R>
__global__ __launch_bounds__(256) void mvm_valu_kernel(int n, const float* __restrict__ px,
                                                       const float* __restrict__ py, float s2,
                                                       const float* __restrict__ V, int ldv, int c0, int jlen,
                                                       float* __restrict__ out, int ldo, int nrhs_total, int direct,
                                                       float amp2, float beta, CgGate gate) {
  if (gate.skip_all()) return;
  __shared__ float sx[kTJ], sy[kTJ];
  __shared__ __attribute__((aligned(16))) float sv[kTJ * NC];
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * (256 * R);
  const int jbeg = blockIdx.y * jlen;
  const int jend = min(n, jbeg + jlen);
  float xi[R], yi[R], acc[R][NC];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = row0 + r * 256 + tid;
    xi[r] = i < n ? px[i] : 0.f;
    yi[r] = i < n ? py[i] : 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[r][c] = 0.f;
  }
  for (int jt = jbeg; jt < jend; jt += kTJ) {
    __syncthreads();
    const int j = jt + tid;
    const bool ok = j < jend;
    sx[tid] = ok ? px[j] : 0.f;
    sy[tid] = ok ? py[j] : 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) sv[tid * NC + c] = ok ? V[(size_t)(c0 + c) * ldv + j] : 0.f;
    __syncthreads();
#pragma unroll 4
    for (int t = 0; t < kTJ; ++t) {
      const float xj = sx[t], yj = sy[t];
      float v[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = sv[t * NC + c];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float dx = xi[r] - xj, dy = yi[r] - yj;
        const float d2 = fmaf(dx, dx, dy * dy);
        const float k = exp2_fast(-(d2 * s2));
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = fmaf(k, v[c], acc[r][c]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = row0 + r * 256 + tid;
    if (i >= n) continue;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (direct) {
        float* y = out + (size_t)(c0 + c) * ldo + i;
        const float res = amp2 * acc[r][c];
        *y = beta != 0.f ? res + beta * *y : res;
      } else {
        out[((size_t)blockIdx.y * nrhs_total + c0 + c) * ldo + i] = acc[r][c];
      }
    }
  }
}

// Y = amp2 * sum_s part[s] + beta * Y, slices summed in order.
__global__ void mvm_reduce_kernel(int n, int nrhs, int S, const float* __restrict__ part, int ldp, float* Y, int ldy,
                                  float amp2, float beta, CgGate gate) {
  if (gate.skip_all()) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  float s = 0.f;
  for (int k = 0; k < S; ++k) s += part[((size_t)k * nrhs + c) * ldp + i];
  float* y = Y + (size_t)c * ldy + i;
  const float res = amp2 * s;
  *y = beta != 0.f ? res + beta * *y : res;
}

template <int NC>
static void launch_valu(const MvmPlan& p, int n, const float* px, const float* py, float s2, const float* V, int ldv,
                        int c0, float* out, int ldo, int nrhs, int direct, float amp2, float beta, CgGate gate,
                        hipStream_t stream) {
  dim3 grid(p.nrb, p.S);
  if (p.R == 4)
    hipLaunchKernelGGL((mvm_valu_kernel<NC, 4>), grid, dim3(256), 0, stream, n, px, py, s2, V, ldv, c0, p.jlen, out,
                       ldo, nrhs, direct, amp2, beta, gate);
  else
    hipLaunchKernelGGL((mvm_valu_kernel<NC, 1>), grid, dim3(256), 0, stream, n, px, py, s2, V, ldv, c0, p.jlen, out,
                       ldo, nrhs, direct, amp2, beta, gate);
}

static size_t valu_workspace(int n, int nrhs) {
  const MvmPlan p = valu_plan(n);
  return p.S > 1 ? align_up(sizeof(float) * (size_t)p.S * nrhs * p.ldp) : 0;
}

size_t valu_mvm_workspace(int n, int nrhs) { return valu_workspace(n, nrhs); }

static int valu_launch(float s2, float amp2, int n, const float* px, const float* py, int nrhs, const float* V,
                       int ldv, float* Y, int ldy, float beta, void* ws, size_t ws_bytes, CgGate gate,
                       hipStream_t stream) {
  const MvmPlan p = valu_plan(n);
  GPL_TRY(check_ws(ws, ws_bytes, valu_workspace(n, nrhs)));
  const bool direct = p.S == 1;
  float* out = direct ? Y : static_cast<float*>(ws);
  const int ldo = direct ? ldy : p.ldp;
  for (int c0 = 0; c0 < nrhs;) {
    const int left = nrhs - c0;
    const int nc = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    hipEvent_t t0 = timing_begin(stream);
    switch (nc) {
      case 16: launch_valu<16>(p, n, px, py, s2, V, ldv, c0, out, ldo, nrhs, direct, amp2, beta, gate, stream); break;
      case 8: launch_valu<8>(p, n, px, py, s2, V, ldv, c0, out, ldo, nrhs, direct, amp2, beta, gate, stream); break;
      case 4: launch_valu<4>(p, n, px, py, s2, V, ldv, c0, out, ldo, nrhs, direct, amp2, beta, gate, stream); break;
      case 2: launch_valu<2>(p, n, px, py, s2, V, ldv, c0, out, ldo, nrhs, direct, amp2, beta, gate, stream); break;
      default: launch_valu<1>(p, n, px, py, s2, V, ldv, c0, out, ldo, nrhs, direct, amp2, beta, gate, stream); break;
    }
    GPL_LAUNCH_CHECK();
    timing_end(t0, stream);
    c0 += nc;
  }
  if (!direct) {
    hipLaunchKernelGGL(mvm_reduce_kernel, dim3(cdiv(n, 256), nrhs), dim3(256), 0, stream, n, nrhs, p.S,
                       static_cast<const float*>(ws), p.ldp, Y, ldy, amp2, beta, gate);
    GPL_LAUNCH_CHECK();
  }
  return GPL_OK;
}

// FP32 form: FMA accumulation on the VALU for a few columns, FP32 MFMA beyond.
static bool fp32_on_mfma(int nrhs) { return nrhs >= kFp32MfmaMinCols; }

size_t mvm_workspace(int n, int nrhs, int prec) {
  if (n <= 0 || nrhs <= 0) return 0;
  if (prec == GPL_PREC_F16X3) return mfma_f16x3_workspace(n, nrhs);
  if (fp32_on_mfma(nrhs)) return mfma_f32_workspace(n, nrhs);
  return valu_workspace(n, nrhs);
}

int mvm_launch(double lengthscale, double amplitude, int n, const float* px, const float* py, int nrhs, const float* V,
               int ldv, float* Y, int ldy, float beta, int prec, void* ws, size_t ws_bytes, CgGate gate,
               hipStream_t stream) {
  const float s2 = (float)kernel_scale2(lengthscale);
  const float amp2 = (float)(amplitude * amplitude);
  if (prec == GPL_PREC_F16X3)
    return mfma_f16x3_launch(s2, amp2, n, px, py, nrhs, V, ldv, Y, ldy, beta, ws, ws_bytes, gate, stream);
  if (fp32_on_mfma(nrhs))
    return mfma_f32_launch(s2, amp2, n, px, py, nrhs, V, ldv, Y, ldy, beta, ws, ws_bytes, gate, stream);
  return valu_launch(s2, amp2, n, px, py, nrhs, V, ldv, Y, ldy, beta, ws, ws_bytes, gate, stream);
}

int check_kernel(const gpl_kernel* k) {
  GPL_REQUIRE(k != nullptr, "kernel is NULL");
  GPL_REQUIRE(k->kind == 0, "kernel kind %d not supported (0 = RBF)", k->kind);
  GPL_REQUIRE(k->lengthscale > 0 && std::isfinite(k->lengthscale), "lengthscale must be > 0");
  GPL_REQUIRE(std::isfinite(k->amplitude), "amplitude must be finite");
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" size_t gpl_gp_kernel_mvm_workspace(int n, int nrhs, int prec) { return mvm_workspace(n, nrhs, prec); }

extern "C" int gpl_gp_kernel_mvm(const gpl_kernel* kern, int n, const float* px, const float* py, int nrhs,
                                 const float* V, int ldv, float* Y, int ldy, float beta, int prec, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
  GPL_TRY(check_kernel(kern));
  GPL_REQUIRE(prec == GPL_PREC_FP32 || prec == GPL_PREC_F16X3, "unknown precision %d", prec);
  GPL_REQUIRE(n >= 0 && nrhs >= 0 && nrhs <= 65535, "n=%d nrhs=%d out of range", n, nrhs);
  if (n == 0 || nrhs == 0) return GPL_OK;
  GPL_REQUIRE(px && py && V && Y, "NULL argument");
  GPL_REQUIRE(ldv >= n && ldy >= n, "ldv=%d ldy=%d must be >= n=%d", ldv, ldy, n);
  GPL_REQUIRE(V != Y, "V and Y must not overlap");
  return mvm_launch(kern->lengthscale, kern->amplitude, n, px, py, nrhs, V, ldv, Y, ldy, beta, prec,
                    ws, ws_bytes, CgGate{}, stream);
}
