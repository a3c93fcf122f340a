// Dense FP64 linear algebra for the preconditioner: a rocBLAS handle per host
// thread and device (its scratch memory always taken from the caller's
// workspace), the inverse and log-determinant of a symmetric positive definite
// matrix by bordering in 64 x 64 blocks, and GEMMs with a long reduction split
// over the device.
#include <cmath>

#include "common.hpp"
#include "dense.hpp"

namespace gpl {

static thread_local rocblas_handle t_handle[16][2] = {};

int blas_handle(rocblas_handle* out, hipStream_t stream, void* scratch, size_t scratch_bytes, int slot) {
  int dev = 0;
  GPL_HIP(hipGetDevice(&dev));
  GPL_REQUIRE(dev >= 0 && dev < 16, "device index %d out of range for the BLAS handles", dev);
  GPL_REQUIRE(slot == 0 || slot == 1, "BLAS handle slot %d", slot);
  rocblas_handle& hs = t_handle[dev][slot];
  if (hs == nullptr) {
    if (rocblas_create_handle(&hs) != rocblas_status_success) {
      hs = nullptr;
      set_error("rocblas_create_handle failed");
      return GPL_EHIP;
    }
  }
  rocblas_handle h = hs;
  if (rocblas_set_stream(h, stream) != rocblas_status_success ||
      rocblas_set_workspace(h, scratch, scratch_bytes) != rocblas_status_success ||
      rocblas_set_pointer_mode(h, rocblas_pointer_mode_host) != rocblas_status_success) {
    set_error("rocblas handle set-up failed");
    return GPL_EHIP;
  }
  *out = h;
  return GPL_OK;
}

struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};
static thread_local SideStream t_side[16];

int side_stream(hipStream_t* s, hipEvent_t ev[3]) {
  int dev = 0;
  GPL_HIP(hipGetDevice(&dev));
  GPL_REQUIRE(dev >= 0 && dev < 16, "device index %d out of range for the side streams", dev);
  SideStream& t = t_side[dev];
  if (t.s == nullptr) {
    GPL_HIP(hipStreamCreateWithFlags(&t.s, hipStreamNonBlocking));
    // the events only order work of two streams on this device: a device-scope
    // release is enough (a system-scope one writes the caches back for the
    // host at every record)
    for (auto& e : t.ev) GPL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence));
  }
  *s = t.s;
  for (int i = 0; i < 3; ++i) ev[i] = t.ev[i];
  return GPL_OK;
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

// out[0] = sum of part[0..n) (one wave, lane-strided then a butterfly: a fixed
// order).
__global__ void fold_sum_kernel(int n, const double* part, double* out) {
  const double s = wave_fold_sum(part, n);
  if (threadIdx.x == 0) *out = s;
}

// One diagonal block of the bordered inverse. S = Gbb + shift I - T from the
// lower triangle of Gbb (T = Y B^T, a 64 x 64 column-major block; null for the
// first block); its Cholesky factor D by four waves in the layout of the block pivot
// (lane a holds row a, wave q the columns [16q, 16q + 16) in registers, every
// wave a copy of the diagonal; one barrier per step, the update vector
// double-buffered by step parity); Dinv = D^{-1} by wave 0 (lane c solves
// column c by forward substitution, the updates of a column's remaining rows
// being independent); S^{-1} = Dinv^T Dinv written over Gbb (both triangles,
// bitwise symmetric); *ld_part = ln|S|. A pivot that is not positive and finite
// sets *info to its global index + 1 (when *info is still 0) and is replaced by
// 1 so that every value stays finite.
constexpr int kSpd = 64;
__global__ __launch_bounds__(256) void spd_block_kernel(double* Gbb, int ldg, double shift,
                                                        const double* __restrict__ T, double* __restrict__ Dinv,
                                                        double* ld_part, int* info, int j0) {
  __shared__ double lv[kSpd][kSpd];      // lv[p][a] = D(a, p) (0 above the diagonal)
  __shared__ double lz[2][kSpd];         // step p: D(a, p) for a > p, else 0
  __shared__ double Di[kSpd][kSpd + 1];  // Di[r][c] = Dinv(r, c)
  __shared__ double idg[kSpd];
  __shared__ double pvs[kSpd];           // the pivots, for ln det after the loop
  // the wave index as a scalar: the owner wave then picks its entry of column p
  // by a register-relative move instead of a chain of selects
  const int a = threadIdx.x & 63, q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b0 = q * 16;
  double s[16];  // s[u] = S(a, b0 + u)
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int b = b0 + u, r = max(a, b), c = min(a, b);
    s[u] = (Gbb[(size_t)c * ldg + r] + (b == a ? shift : 0.0)) - (T ? T[(size_t)c * kSpd + r] : 0.0);
  }
  double dg = (Gbb[(size_t)a * ldg + a] + shift) - (T ? T[(size_t)a * kSpd + a] : 0.0);
  int bad = -1;
  for (int p = 0; p < kSpd; ++p) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)__double_as_longlong(dg), p);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)__double_as_longlong(dg) >> 32), p);
    const double dpp = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    const bool ok = dpp > 0.0 && isfinite(dpp);
    if (!ok && bad < 0) bad = p;
    const double pv = ok ? dpp : 1.0;
    if (threadIdx.x == 0) pvs[p] = pv;  // ln D(p, p)^2 is summed after the loop
    const int buf = p & 1;
    if (q == p / 16) {  // this wave holds column p
      const double sp = s[p - b0];
      const double r = rsqrt_f64(pv), lpp = pv * r;
      const double l = a == p ? lpp : (a > p ? sp * r : 0.0);
      lv[p][a] = l;
      lz[buf][a] = a > p ? l : 0.0;
    }
    __syncthreads();
    const double la = lz[buf][a];
#pragma unroll
    for (int u = 0; u < 16; ++u) s[u] -= la * lz[buf][b0 + u];
    dg -= la * la;
  }
  if (threadIdx.x < kSpd) idg[threadIdx.x] = 1.0 / lv[threadIdx.x][threadIdx.x];
  __syncthreads();
  // sum over the pivots of ln D(p, p)^2: one logarithm a lane, a fixed-order
  // butterfly over the wave
  const double lsum = q == 0 ? warp_sum(log(pvs[a])) : 0.0;
  if (q == 0) {
    double x[kSpd];
#pragma unroll
    for (int r = 0; r < kSpd; ++r) x[r] = r == a ? 1.0 : 0.0;
#pragma unroll
    for (int r = 0; r < kSpd; ++r) {
      x[r] *= idg[r];
#pragma unroll
      for (int w = r + 1; w < kSpd; ++w) x[w] = fma(-lv[r][w], x[r], x[w]);
    }
#pragma unroll
    for (int r = 0; r < kSpd; ++r) {
      Di[r][a] = x[r];
      Dinv[(size_t)a * kSpd + r] = x[r];
    }
  }
  __syncthreads();
  double acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.0;
  for (int r = 0; r < kSpd; ++r) {
    const double xa = Di[r][a];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = fma(xa, Di[r][b0 + u], acc[u]);
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) Gbb[(size_t)(b0 + u) * ldg + a] = acc[u];
  if (threadIdx.x == 0) {
    *ld_part = lsum;
    if (bad >= 0 && *info == 0) *info = j0 + bad + 1;
  }
}

int border_begin(int* info, hipStream_t stream) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, stream, info, 0);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int border_step(rocblas_handle h, double* G, int ldg, int j0, double shift, const SpdScratch& w, int* info,
                hipStream_t stream) {
  GPL_REQUIRE(j0 >= 0 && j0 % kSpd == 0, "block start %d must be a multiple of %d", j0, kSpd);
  const double one = 1.0, minus_one = -1.0, zero = 0.0;
  const auto N = rocblas_operation_none, Tr = rocblas_operation_transpose;
  double* Gb = G + j0;                      // Ginv[b, :b]
  double* Gbb = G + (size_t)j0 * ldg + j0;  // G[b, b], then Ginv[b, b]
  double* Gcol = G + (size_t)j0 * ldg;      // G[:b, b] = G[b, :b]^T (read), then Ginv[:b, b]
  if (j0 > 0) {
    // Y = G[b, :b] Ginv[:b, :b];  T = Y G[b, :b]^T = G[b, :b] Ginv G[b, :b]^T
    GPL_TRY(split_gemm(h, Tr, N, kSpd, j0, j0, std::max(1, std::min(16, j0 / 256)), 1.0, Gcol, ldg, G, ldg, 0.0, w.Y,
                       kSpd, w.split, w.split_elems, stream));
    GPL_TRY(split_gemm(h, N, N, kSpd, kSpd, j0, std::max(1, j0 / 64), 1.0, w.Y, kSpd, Gcol, ldg, 0.0, w.T, kSpd,
                       w.split, w.split_elems, stream));
  }
  hipLaunchKernelGGL(spd_block_kernel, dim3(1), dim3(256), 0, stream, Gbb, ldg, shift, j0 > 0 ? w.T : nullptr,
                     w.Dinv, w.ld_part + j0 / kSpd, info, j0);
  GPL_LAUNCH_CHECK();
  if (j0 > 0) {
    // W = Dinv Y; Ginv[:b, :b] += W^T W (= Y^T S^{-1} Y); Ginv[b, :b] = -Dinv^T W (= -S^{-1} Y) and its transpose
    if (rocblas_dgemm(h, N, N, kSpd, j0, kSpd, &one, w.Dinv, kSpd, w.Y, kSpd, &zero, w.W, kSpd) !=
            rocblas_status_success ||
        rocblas_dgemm(h, Tr, N, j0, j0, kSpd, &one, w.W, kSpd, w.W, kSpd, &one, G, ldg) != rocblas_status_success ||
        rocblas_dgemm(h, Tr, N, kSpd, j0, kSpd, &minus_one, w.Dinv, kSpd, w.W, kSpd, &zero, Gb, ldg) !=
            rocblas_status_success ||
        rocblas_dgemm(h, Tr, N, j0, kSpd, kSpd, &minus_one, w.W, kSpd, w.Dinv, kSpd, &zero, Gcol, ldg) !=
            rocblas_status_success) {
      set_error("rocblas_dgemm (bordered inverse, block at %d) failed", j0);
      return GPL_EHIP;
    }
  }
  return GPL_OK;
}

int border_finish(int k, const SpdScratch& w, double* logdet, hipStream_t stream) {
  hipLaunchKernelGGL(fold_sum_kernel, dim3(1), dim3(64), 0, stream, k / kSpd, w.ld_part, logdet);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

// C (m x n, ld ldc) = alpha * sum_s Wp[s] + beta C, the splits in order; the
// beta term's C(r, c) is Cf[r * n + c] widened when Cf is set.
__global__ void split_sum_kernel(int m, int n, int nsplit, const double* __restrict__ Wp, double alpha, double beta,
                                 double* C, int ldc, const float* __restrict__ Cf) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int r = e % m, c = e / m;
  double* y = C + (size_t)c * ldc + r;
  // issued ahead of the split loads
  const double y0 = beta == 0.0 ? 0.0 : (Cf ? (double)Cf[(size_t)r * n + c] : *y);
  // in split order; the loads of each group of 8 splits are issued together
  // (past the last split a load repeats it, at a valid address, and is not added)
  double v = 0.0;
  const size_t mn = (size_t)m * n;
  for (int s0 = 0; s0 < nsplit; s0 += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = Wp[(size_t)min(s0 + u, nsplit - 1) * mn + e];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (s0 + u < nsplit) v += t[u];
  }
  *y = beta == 0.0 ? alpha * v : alpha * v + beta * y0;
}

size_t split_gemm_scratch(int m, int n, int nsplit) { return (size_t)nsplit * m * n * sizeof(double); }

int split_gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int kdim, int nsplit,
               double alpha, const double* A, int lda, const double* B, int ldb, double beta, double* C, int ldc,
               double* scratch, size_t scratch_elems, hipStream_t stream, const float* Cf) {
  const size_t per = (size_t)m * n;
  GPL_REQUIRE(m > 0 && n > 0 && kdim > 0, "split product of empty size");
  GPL_REQUIRE(scratch_elems >= per, "split product scratch holds %zu doubles, one split needs %zu", scratch_elems,
              per);
  const size_t fit = scratch_elems / per;
  nsplit = std::max(1, std::min(std::min(nsplit, kdim), (int)std::min<size_t>(fit, 1 << 20)));
  const int kc = cdiv(kdim, nsplit);
  nsplit = cdiv(kdim, kc);
  const int last = kdim - (nsplit - 1) * kc;  // rows of the reduction in the last split
  // element (i, l) of op(A) is A[l*lda + i] without transpose, A[i*lda + l] with it:
  // a split of the reduction index l moves A by kc columns (no transpose) or
  // kc rows (transpose); likewise for B with (l, j)
  const rocblas_stride sa = ta == rocblas_operation_none ? (rocblas_stride)kc * lda : kc;
  const rocblas_stride sb = tb == rocblas_operation_none ? kc : (rocblas_stride)kc * ldb;
  const double one = 1.0, zero = 0.0;
  // splits of kc rows in one batched call; a shorter last split in a call of its own
  const int nfull = last == kc ? nsplit : nsplit - 1;
  if (nfull > 1 &&
      rocblas_dgemm_strided_batched(h, ta, tb, m, n, kc, &one, A, lda, sa, B, ldb, sb, &zero, scratch, m,
                                    (rocblas_stride)m * n, nfull) != rocblas_status_success) {
    set_error("rocblas_dgemm_strided_batched failed");
    return GPL_EHIP;
  }
  const int one_from = nfull > 1 ? nfull : 0;  // splits [one_from, nsplit) by plain calls
  for (int s = one_from; s < nsplit; ++s)
    if (rocblas_dgemm(h, ta, tb, m, n, s == nsplit - 1 ? last : kc, &one, A + (size_t)s * sa, lda, B + (size_t)s * sb,
                      ldb, &zero, scratch + (size_t)s * m * n, m) != rocblas_status_success) {
    set_error("rocblas_dgemm (split %d of %d) failed", s, nsplit);
    return GPL_EHIP;
  }
  hipLaunchKernelGGL(split_sum_kernel, dim3(cdiv(m * n, 256)), dim3(256), 0, stream, m, n, nsplit, scratch, alpha,
                     beta, C, ldc, Cf);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl
