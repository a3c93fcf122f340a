// Matrix-free kernel-matrix product Y = K V + beta Y with the RBF kernel of
// Sec. 3.1 (eq. "grbf"), K_ij = a^2 exp(-|p_i - p_j|^2 / (2 l^2)). The paper
// forms this product on the fly, never storing K (Sec. 3.3, transmission
// matrix "too large to store"); here the same holds on gfx950.
//
// A product is prepared once per point set (the tile plan: sorted points,
// chunk boxes and the lists of chunk pairs that can be non-zero) and then run
// for any number of right-hand-side blocks; the CG driver prepares once per
// solve. Both precision forms run on MFMA (mvm_mfma.hip).
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"
#include "mvm_mfma.hpp"

namespace gpl {

template <class C>
static void carve_mvm(C& cv, int n, int nrhs, int prec, TilePlan* plan, void** scratch, size_t* scratch_bytes) {
  TilePlan p;
  plan_carve(cv, n, p);
  const size_t sb = mfma_workspace(n, nrhs, prec);
  char* s = cv.template take<char>(sb);
  if (plan) *plan = p;
  if (scratch) *scratch = s;
  if (scratch_bytes) *scratch_bytes = sb;
}

size_t mvm_workspace(int n, int nrhs, int prec) {
  if (n <= 0 || nrhs <= 0) return 0;
  Sizer s;
  carve_mvm(s, n, nrhs, prec, nullptr, nullptr, nullptr);
  return s.used;
}

int mvm_prepare(MvmCtx& m, double lengthscale, double amplitude, int n, const float* px, const float* py,
                const gpl_grid* grid, int nrhs, int prec, void* ws, size_t ws_bytes, hipStream_t stream) {
  GPL_TRY(check_ws(ws, ws_bytes, mvm_workspace(n, nrhs, prec)));
  Carver cv(ws, ws_bytes);
  void* scratch;
  size_t scratch_bytes;
  carve_mvm(cv, n, nrhs, prec, &m.plan, &scratch, &scratch_bytes);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  GPL_TRY(mfma_carve(m.plan, prec, nrhs, scratch, scratch_bytes, m.bufs));
  m.prec = prec;
  m.nrhs_max = nrhs;
  m.s2 = (float)kernel_scale2(lengthscale);
  m.amp2 = (float)(amplitude * amplitude);
  GPL_TRY(mfma_zero_rhs(m.bufs, prec, stream));
  return plan_build(m.plan, n, px, py, grid, m.s2, plan_threshold(prec), plan_lo_threshold(prec), stream);
}

int mvm_run_prepared(const MvmCtx& m, int nrhs, float* Y, int ldy, float beta, CgGate gate, hipStream_t stream) {
  GPL_REQUIRE(nrhs <= m.nrhs_max, "product prepared for %d columns, %d given", m.nrhs_max, nrhs);
  return mfma_product(m.plan, m.bufs, m.prec, m.s2, m.amp2, nrhs, Y, ldy, beta, gate, stream);
}

int mvm_run(const MvmCtx& m, int nrhs, const float* V, int ldv, float* Y, int ldy, float beta, CgGate gate,
            hipStream_t stream) {
  GPL_REQUIRE(nrhs <= m.nrhs_max, "product prepared for %d columns, %d given", m.nrhs_max, nrhs);
  GPL_TRY(mfma_prep_rhs(m.plan, m.bufs, m.prec, nrhs, V, ldv, gate, stream));
  return mvm_run_prepared(m, nrhs, Y, ldy, beta, gate, stream);
}

int mvm_launch(double lengthscale, double amplitude, int n, const float* px, const float* py, const gpl_grid* grid,
               int nrhs, const float* V, int ldv, float* Y, int ldy, float beta, int prec, void* ws, size_t ws_bytes,
               CgGate gate, hipStream_t stream) {
  MvmCtx m;
  GPL_TRY(mvm_prepare(m, lengthscale, amplitude, n, px, py, grid, nrhs, prec, ws, ws_bytes, stream));
  return mvm_run(m, nrhs, V, ldv, Y, ldy, beta, gate, stream);
}

// out[0] = listed (row tile, chunk) pairs, out[1] = listed (subtile, chunk) pairs.
__global__ void plan_live_sum_kernel(int nrt, int nch, const int* count, const uint32_t* list, long long* out) {
  __shared__ long long red[3][4];
  long long u = 0, t = 0, l = 0;
  for (int r = blockIdx.x; r < nrt; r += gridDim.x) {
    if (threadIdx.x == 0) u += count[r];
    for (int k = threadIdx.x; k < count[r]; k += blockDim.x) {
      const uint32_t e = list[(size_t)r * nch + k];
      t += __popc(entry_mask(e));
      l += __popc(entry_lomask(e));
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    u += __shfl_xor(u, off, 64);
    t += __shfl_xor(t, off, 64);
    l += __shfl_xor(l, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = u;
    red[1][threadIdx.x >> 6] = t;
    red[2][threadIdx.x >> 6] = l;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) out[q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
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

namespace gpl {

// The windowed kernel (kind 1) as a Gaussian product over the grid's points
// with their pixel shapes, Z staged at the start of the workspace.
int windowed_mvm(const gpl_kernel* kern, const gpl_grid* grid, int n, const float* px, const float* py, int nrhs,
                 const float* V, int ldv, float* Y, int ldy, float beta, void* ws, size_t ws_bytes,
                 hipStream_t stream) {
  GPL_REQUIRE(grid != nullptr, "the windowed kernel (kind 1) needs the grid of the points");
  GPL_REQUIRE((long)grid->n * grid->ss * grid->n * grid->ss == n, "grid does not match n=%d", n);
  GPL_TRY(check_ws(ws, ws_bytes, (size_t)3 * n * sizeof(float)));
  float* z = static_cast<float*>(ws);
  GPL_TRY(pixel_shapes_launch(grid->n * grid->ss, px, py, z, stream));
  const double l2 = kern->lengthscale * kern->lengthscale;
  const GSide side{px, py, z, nullptr, n};
  return gauss_product_launch(side, side, l2, kern->amplitude * kern->amplitude * l2, nrhs, V, ldv, Y, ldy, beta,
                              stream);
}

int check_kernel_any(const gpl_kernel* k) {
  GPL_REQUIRE(k != nullptr, "kernel is NULL");
  GPL_REQUIRE(k->kind == 0 || k->kind == 1, "kernel kind %d not supported (0 = RBF, 1 = windowed)", k->kind);
  GPL_REQUIRE(k->lengthscale > 0 && std::isfinite(k->lengthscale), "lengthscale must be > 0");
  GPL_REQUIRE(std::isfinite(k->amplitude), "amplitude must be finite");
  return GPL_OK;
}

}  // namespace gpl

extern "C" int gpl_gp_kernel_mvm(const gpl_kernel* kern, const gpl_grid* grid, int n, const float* px,
                                 const float* py, int nrhs, const float* V, int ldv, float* Y, int ldy, float beta,
                                 int prec, void* ws, size_t ws_bytes, hipStream_t stream) {
  GPL_TRY(check_kernel_any(kern));
  if (kern->kind == 1) {
    if (prec != GPL_PREC_FP32) {
      set_error("the windowed kernel (kind 1) runs in the FP32 form only");
      return GPL_EUNSUPPORTED;
    }
    GPL_REQUIRE(n >= 0 && nrhs >= 0 && nrhs <= 65535, "n=%d nrhs=%d out of range", n, nrhs);
    if (n == 0 || nrhs == 0) return GPL_OK;
    GPL_REQUIRE(px && py && V && Y, "NULL argument");
    GPL_REQUIRE(ldv >= n && ldy >= n, "ldv=%d ldy=%d must be >= n=%d", ldv, ldy, n);
    GPL_REQUIRE(V != Y, "V and Y must not overlap");
    return windowed_mvm(kern, grid, n, px, py, nrhs, V, ldv, Y, ldy, beta, ws, ws_bytes, stream);
  }
  GPL_REQUIRE(prec == GPL_PREC_FP32 || prec == GPL_PREC_F16X3, "unknown precision %d", prec);
  GPL_REQUIRE(n >= 0 && nrhs >= 0 && nrhs <= 65535, "n=%d nrhs=%d out of range", n, nrhs);
  if (n == 0 || nrhs == 0) return GPL_OK;
  GPL_REQUIRE(px && py && V && Y, "NULL argument");
  GPL_REQUIRE(ldv >= n && ldy >= n, "ldv=%d ldy=%d must be >= n=%d", ldv, ldy, n);
  GPL_REQUIRE(V != Y, "V and Y must not overlap");
  if (grid) {
    GPL_REQUIRE(grid->n >= 1 && grid->ss >= 1, "bad grid");
    GPL_REQUIRE((long)grid->n * grid->ss * grid->n * grid->ss == n, "grid has %ld fine points, n=%d",
                (long)grid->n * grid->ss * grid->n * grid->ss, n);
  }
  return mvm_launch(kern->lengthscale, kern->amplitude, n, px, py, grid, nrhs, V, ldv, Y, ldy, beta, prec, ws,
                    ws_bytes, CgGate{}, stream);
}

extern "C" size_t gpl_gp_kernel_mvm_plan_workspace(int n) {
  return n > 0 ? align_up(plan_workspace(n)) + 2 * kAlign : 0;
}

extern "C" int gpl_gp_kernel_mvm_plan_stats(const gpl_kernel* kern, const gpl_grid* grid, int n, const float* px,
                                            const float* py, int prec, long long* live_tiles,
                                            long long* live_subtiles, long long* live_lo, void* ws,
                                            size_t ws_bytes, hipStream_t stream) {
  GPL_TRY(check_kernel(kern));
  GPL_REQUIRE(prec == GPL_PREC_FP32 || prec == GPL_PREC_F16X3, "unknown precision %d", prec);
  GPL_REQUIRE(n >= 1 && px && py && live_tiles, "bad arguments");
  if (grid)
    GPL_REQUIRE((long)grid->n * grid->ss * grid->n * grid->ss == n, "grid does not match n=%d", n);
  GPL_TRY(check_ws(ws, ws_bytes, gpl_gp_kernel_mvm_plan_workspace(n)));
  Carver cv(ws, ws_bytes);
  TilePlan p;
  plan_carve(cv, n, p);
  long long* dsum = cv.take<long long>(3);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  GPL_TRY(plan_build(p, n, px, py, grid, (float)kernel_scale2(kern->lengthscale), plan_threshold(prec),
                     plan_lo_threshold(prec), stream));
  hipLaunchKernelGGL(plan_live_sum_kernel, dim3(1), dim3(256), 0, stream, p.nrt, p.nch, p.count, p.list, dsum);
  GPL_LAUNCH_CHECK();
  long long h[3];
  GPL_HIP(hipMemcpyAsync(h, dsum, sizeof(h), hipMemcpyDeviceToHost, stream));
  GPL_HIP(hipStreamSynchronize(stream));
  *live_tiles = h[0];
  if (live_subtiles) *live_subtiles = h[1];
  if (live_lo) *live_lo = h[2];
  return GPL_OK;
}
