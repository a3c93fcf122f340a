// Conjugate gradients on A X = B with A = B_op K B_op^T + sigma^2 I, one
// independent recurrence per right-hand-side column, all columns sharing each
// application of A (the evidence of Sec. 3.1, eq. "gp-mll", evaluated with CG
// as discussed in Sec. 3.3). Vectors are FP32; every dot product, the alpha and
// beta recurrences and the recorded Lanczos coefficients are FP64.
//
// One iteration is a fixed sequence of launches on the caller's stream:
//   B_op^T P (written straight into the kernel product's RHS buffers)
//   -> T2 = K B_op^T P  ->  AP = B_op T2 + sigma^2 P  (+ p.Ap partials)
//   -> update1 (alpha; X += alpha P; R -= alpha AP; r.r partials)
//   -> update2 (beta; P = R + beta P; bookkeeping; partial max |P| for the
//      column scales of the precision form).
// Per-column state is double-buffered by iteration parity so that every block
// of a kernel reads the same old values. Kernels return at once when no column
// is active. Either every iteration up to the cap is enqueued at once (fully
// asynchronous), or the host enqueues iterations in chunks, keeps one chunk in
// flight ahead, and after each chunk reads the number of active columns from a
// small coherent host buffer written by a snapshot kernel (waiting on an event,
// never synchronising the device). After the last iteration one more product
// with A gives the true residual b - A x of the returned iterate.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "internal.hpp"

namespace gpl {

struct CgBuffers {
  float *R, *P, *AP, *T2;
  int ldv, ldf;
  void* mvm_ws;
  size_t mvm_ws_bytes;
  double *pap_part, *rr_part;
  int ntiles, nb_upd;
  ColState* st[2];
  double* bb;
  int* n_active;  // [2]
  unsigned* pmax;  // [nrhs][nb_upd] partial max |P| (float bits)
};

template <class C>
static void carve_cg(C& c, int npix, int N, int nrhs, int prec, CgBuffers* b, size_t* mvm_bytes_out, int ss, int n) {
  const int ldv = round_up(npix, 64), ldf = round_up(N, 64);
  const size_t mvm_bytes = mvm_workspace(N, nrhs, prec);
  const int ntiles = psf_forward_tiles(n, ss), nb_upd = cg_blocks(npix);
  float* R = c.template take<float>((size_t)ldv * nrhs);
  float* P = c.template take<float>((size_t)ldv * nrhs);
  float* AP = c.template take<float>((size_t)ldv * nrhs);
  float* T2 = c.template take<float>((size_t)ldf * nrhs);
  char* mws = c.template take<char>(mvm_bytes);
  double* pap = c.template take<double>((size_t)ntiles * nrhs);
  double* rrp = c.template take<double>((size_t)nb_upd * nrhs);
  ColState* s0 = c.template take<ColState>(nrhs);
  ColState* s1 = c.template take<ColState>(nrhs);
  double* bb = c.template take<double>(nrhs);
  int* na = c.template take<int>(2);
  unsigned* pm = c.template take<unsigned>((size_t)nb_upd * nrhs);
  if (b) {
    *b = CgBuffers{R, P, AP, T2, ldv, ldf, mws, mvm_bytes, pap, rrp, ntiles, nb_upd, {s0, s1}, bb, na, pm};
  }
  if (mvm_bytes_out) *mvm_bytes_out = mvm_bytes;
}

// Block maximum of v >= 0 (result in thread 0).
__device__ __forceinline__ float block_max(float v, float* smem) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) smem[threadIdx.x >> 6] = v;
  __syncthreads();
  float m = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, smem[w]);
  return m;
}

// R = P = B, X = 0, partial |b|^2 and partial max |P|.
__global__ __launch_bounds__(256) void cg_init_kernel(int npix, const float* __restrict__ Bm, int ldb, float* X,
                                                      int ldx, float* R, float* P, int ldv, double* part, int nb,
                                                      unsigned* pmax) {
  __shared__ double red[4];
  __shared__ float redm[4];
  const int c = blockIdx.y;
  double s = 0.0;
  float m = 0.f;
#pragma unroll
  for (int e = 0; e < kUpdPer; ++e) {
    const int i = blockIdx.x * kUpdSpan + e * 256 + threadIdx.x;
    if (i < npix) {
      const float b = Bm[(size_t)c * ldb + i];
      R[(size_t)c * ldv + i] = b;
      P[(size_t)c * ldv + i] = b;
      X[(size_t)c * ldx + i] = 0.f;
      s += (double)b * b;
      m = fmaxf(m, fabsf(b));
    }
  }
  s = block_sum_double(s, red);
  m = block_max(m, redm);
  if (threadIdx.x == 0) {
    part[(size_t)c * nb + blockIdx.x] = s;
    pmax[(size_t)c * nb + blockIdx.x] = __float_as_uint(m);
  }
}

__global__ void cg_init_state_kernel(int nrhs, const double* part, int nb, ColState* st0, ColState* st1, double* bb,
                                     int* n_active, int limit) {
  // one thread per column; thread 0 of the block also writes the active count
  __shared__ int count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < nrhs; c += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)c * nb + b];
    ColState z;
    z.rr = s;
    z.alpha = 0.0;
    z.iters = 0;
    z.bad = 0;
    if (!isfinite(s)) {
      z.status = GPL_CG_NONFINITE;
      z.active = 0;
    } else if (s == 0.0 || limit == 0) {
      z.status = s == 0.0 ? GPL_CG_CONVERGED : GPL_CG_MAXITER;
      z.active = 0;
    } else {
      z.status = GPL_CG_CONVERGED;
      z.active = 1;
    }
    st0[c] = z;
    st1[c] = z;
    bb[c] = s;
    if (z.active) atomicAdd(&count, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    n_active[0] = count;
    n_active[1] = count;
  }
}

// alpha = rr / pAp (redundantly in every block, fixed order), X += alpha P,
// R -= alpha AP, partial r.r of the new residual.
__device__ __forceinline__ void cg_update1_body(int bx, int c, int npix, float* X, int ldx, float* R,
                                                const float* P, const float* AP, int ldv, const double* pap_part,
                                                int ntiles, double* rr_part, int nb, const ColState* sin,
                                                ColState* sout, const int* n_active_in, int* n_active_out) {
  __shared__ double red[4];
  __shared__ double s_alpha;
  __shared__ int s_ok;
  if (bx == 0 && c == 0 && threadIdx.x == 0) *n_active_out = 0;
  // this thread's vector entries and the p.Ap partials, loaded before the gate
  // is read (always in bounds; unused when the column has stopped) so that the
  // round trips overlap
  int i[kUpdPer];
  float xv[kUpdPer], pv[kUpdPer], apv[kUpdPer], rv[kUpdPer];
#pragma unroll
  for (int e = 0; e < kUpdPer; ++e) {
    i[e] = bx * kUpdSpan + e * 256 + threadIdx.x;
    const int ic = min(i[e], npix - 1);
    const size_t iv = (size_t)c * ldv + ic;
    xv[e] = X[(size_t)c * ldx + ic];
    pv[e] = P[iv];
    apv[e] = AP[iv];
    rv[e] = R[iv];
  }
  const double pap = threadIdx.x < 64 ? wave_fold_sum(pap_part + (size_t)c * ntiles, ntiles) : 0.0;
  if (*n_active_in == 0) return;
  const ColState st = sin[c];
  if (!st.active) return;
  if (threadIdx.x == 0) {
    const double a = st.rr / pap;
    const int ok = (pap > 0.0) && isfinite(a);
    s_alpha = ok ? a : 0.0;
    s_ok = ok;
    if (bx == 0) {
      sout[c].alpha = s_alpha;
      sout[c].bad = ok ? 0 : (isfinite(pap) ? 1 : 2);
    }
  }
  __syncthreads();
  const double alpha = s_alpha;
  double s = 0.0;
  if (s_ok) {
    const float af = (float)alpha;
#pragma unroll
    for (int e = 0; e < kUpdPer; ++e)
      if (i[e] < npix) {
        X[(size_t)c * ldx + i[e]] = fmaf(af, pv[e], xv[e]);
        const float r = fmaf(-af, apv[e], rv[e]);
        R[(size_t)c * ldv + i[e]] = r;
        s += (double)r * r;
      }
  }
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) rr_part[(size_t)c * nb + bx] = s;
}

__global__ __launch_bounds__(256) void cg_update1_kernel(int npix, float* X, int ldx, float* R, const float* P,
                                                         const float* AP, int ldv, const double* pap_part,
                                                         int ntiles, double* rr_part, int nb, const ColState* sin,
                                                         ColState* sout, const int* n_active_in,
                                                         int* n_active_out) {
  cg_update1_body(blockIdx.x, blockIdx.y, npix, X, ldx, R, P, AP, ldv, pap_part, ntiles, rr_part, nb, sin, sout,
                  n_active_in, n_active_out);
}

// beta = rr_new / rr, P = R + beta P; block 0 of each column records the Lanczos
// coefficients and decides the column's status for the next iteration.
__device__ __forceinline__ void cg_update2_body(int bx, int c, int npix, const float* R, float* P, int ldv,
                                                const double* rr_part, int nb, const ColState* sin, ColState* sout,
                                                const double* bb, const int* n_active_in, int* n_active_out,
                                                double tol, int max_iter, int fixed_iters, int n_lanczos,
                                                double* ab, unsigned* pmax) {
  __shared__ double s_beta;
  __shared__ int s_go;
  __shared__ float redm[4];
  // this thread's vector entries and the r.r partials, loaded before the gate
  // is read (always in bounds; unused when the column has stopped)
  int i[kUpdPer];
  float rv[kUpdPer], pv[kUpdPer];
#pragma unroll
  for (int e = 0; e < kUpdPer; ++e) {
    i[e] = bx * kUpdSpan + e * 256 + threadIdx.x;
    const size_t iv = (size_t)c * ldv + min(i[e], npix - 1);
    rv[e] = R[iv];
    pv[e] = P[iv];
  }
  const double rr_new = threadIdx.x < 64 ? wave_fold_sum(rr_part + (size_t)c * nb, nb) : 0.0;
  const ColState st = sin[c];
  if (*n_active_in == 0 || !st.active) {  // carry the state into the other parity
    if (bx == 0 && threadIdx.x == 0) sout[c] = st;
    return;
  }
  if (threadIdx.x == 0) {
    const ColState half = sout[c];  // alpha and bad written by update1
    const double beta = rr_new / st.rr;
    ColState nx;
    nx.alpha = half.alpha;
    nx.bad = 0;
    nx.iters = st.iters;
    nx.rr = st.rr;
    nx.status = GPL_CG_CONVERGED;
    nx.active = 0;
    int go = 0;
    if (half.bad) {
      nx.status = half.bad == 1 ? GPL_CG_BREAKDOWN : GPL_CG_NONFINITE;
    } else if (!isfinite(rr_new) || !isfinite(beta)) {
      nx.status = GPL_CG_NONFINITE;
      nx.iters = st.iters + 1;
    } else {
      go = 1;
      nx.rr = rr_new;
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
#pragma unroll
  for (int e = 0; e < kUpdPer; ++e)
    if (i[e] < npix) {
      const float pn = fmaf((float)s_beta, pv[e], rv[e]);
      P[(size_t)c * ldv + i[e]] = pn;
      m = fmaxf(m, fabsf(pn));
    }
  m = block_max(m, redm);
  if (threadIdx.x == 0) pmax[(size_t)c * nb + bx] = __float_as_uint(m);
}

__global__ __launch_bounds__(256) void cg_update2_kernel(int npix, const float* R, float* P, int ldv,
                                                         const double* rr_part, int nb, const ColState* sin,
                                                         ColState* sout, const double* bb, const int* n_active_in,
                                                         int* n_active_out, double tol, int max_iter,
                                                         int fixed_iters, int n_lanczos, double* ab,
                                                         unsigned* pmax) {
  cg_update2_body(blockIdx.x, blockIdx.y, npix, R, P, ldv, rr_part, nb, sin, sout, bb, n_active_in, n_active_out, tol,
                  max_iter, fixed_iters, n_lanczos, ab, pmax);
}

// ---- grouped launches (serving): workgroup (local % nb, local / nb) of slot s.
__global__ __launch_bounds__(256) void cg_update1_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  const int local = blockIdx.x - B.off[s];
  cg_update1_body(local % S.nb_upd, local / S.nb_upd, S.npix, S.X, S.ldv, S.R, S.P, S.AP, S.ldv, S.pap_part,
                  S.ntiles_fwd, S.rr_part, S.nb_upd, S.st[p], S.st[1 - p], S.n_active + p, S.n_active + (1 - p));
}

__global__ __launch_bounds__(256) void cg_update2_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  const int local = blockIdx.x - B.off[s];
  cg_update2_body(local % S.nb_upd, local / S.nb_upd, S.npix, S.R, S.P, S.ldv, S.rr_part, S.nb_upd, S.st[p],
                  S.st[1 - p], S.bb, S.n_active + p, S.n_active + (1 - p), S.tol, S.max_iter, 0, S.n_lanczos, S.ab,
                  S.pmax);
}

// Partial max |X| per block (float bits), for the column scales of the
// precision form when A is applied to the iterate itself.
__global__ __launch_bounds__(256) void cg_absmax_kernel(int npix, const float* __restrict__ X, int ldx,
                                                        unsigned* pmax, int nb) {
  __shared__ float redm[4];
  const int c = blockIdx.y;
  float m = 0.f;
#pragma unroll
  for (int e = 0; e < kUpdPer; ++e) {
    const int i = blockIdx.x * kUpdSpan + e * 256 + threadIdx.x;
    if (i < npix) m = fmaxf(m, fabsf(X[(size_t)c * ldx + i]));
  }
  m = block_max(m, redm);
  if (threadIdx.x == 0) pmax[(size_t)c * nb + blockIdx.x] = __float_as_uint(m);
}

// Partial |b - A x|^2 per block, in FP64.
__global__ __launch_bounds__(256) void cg_true_residual_kernel(int npix, const float* __restrict__ Bm, int ldb,
                                                               const float* __restrict__ AX, int ldv,
                                                               double* part, int nb) {
  __shared__ double red[4];
  const int c = blockIdx.y;
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < kUpdPer; ++e) {
    const int i = blockIdx.x * kUpdSpan + e * 256 + threadIdx.x;
    if (i < npix) {
      const double d = (double)Bm[(size_t)c * ldb + i] - (double)AX[(size_t)c * ldv + i];
      s += d * d;
    }
  }
  s = block_sum_double(s, red);
  if (threadIdx.x == 0) part[(size_t)c * nb + blockIdx.x] = s;
}

// true_relres[c] = |b - A x| / |b| from the partials, in block order.
__global__ void cg_true_residual_fold_kernel(int nrhs, const double* part, int nb, const double* bb,
                                             double* true_relres) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)c * nb + b];
  true_relres[c] = bb[c] > 0.0 ? sqrt(s / bb[c]) : sqrt(s);
}

__global__ void cg_snapshot_kernel(const int* n_active, volatile int* host_flag) {
  if (threadIdx.x == 0) {
    *host_flag = *n_active;
    __threadfence_system();
  }
}

__global__ void cg_finalize_kernel(int nrhs, const ColState* st, const double* bb, double* bnorm2, int* iters,
                                   double* relres, int* status, int n_lanczos, double* ab) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const ColState s = st[c];
  if (bnorm2) bnorm2[c] = bb[c];
  if (iters) iters[c] = s.iters;
  if (relres) relres[c] = bb[c] > 0.0 ? sqrt(s.rr / bb[c]) : 0.0;
  if (status) status[c] = s.active ? GPL_CG_MAXITER : s.status;
  // zero the Lanczos slots beyond the column's count
  if (ab)
    for (int k = s.iters; k < n_lanczos; ++k) {
      ab[((size_t)c * n_lanczos + k) * 2 + 0] = 0.0;
      ab[((size_t)c * n_lanczos + k) * 2 + 1] = 0.0;
    }
}

int cg_update_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                      hipStream_t stream) {
  SlotBatch B;
  B.nslots = nslots;
  B.off[0] = 0;
  for (int s = 0; s < nslots; ++s) {
    B.slot[s] = dslots[s];
    B.off[s + 1] = B.off[s] + hslots[s]->nb_upd * hslots[s]->nrhs;
  }
  if (B.off[nslots] == 0) return GPL_OK;
  hipLaunchKernelGGL(cg_update1_grouped_kernel, dim3(B.off[nslots]), dim3(256), 0, stream, B, p);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(cg_update2_grouped_kernel, dim3(B.off[nslots]), dim3(256), 0, stream, B, p);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int cg_init_launch(int npix, int nrhs, const float* Bm, int ldb, float* X, int ldx, float* R, float* P, int ldv,
                   double* part, ColState* st0, ColState* st1, double* bb, int* n_active, int limit, unsigned* pmax,
                   hipStream_t stream) {
  const int nb = cg_blocks(npix);
  hipLaunchKernelGGL(cg_init_kernel, dim3(nb, nrhs), dim3(256), 0, stream, npix, Bm, ldb, X, ldx, R, P, ldv, part, nb,
                     pmax);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(cg_init_state_kernel, dim3(1), dim3(256), 0, stream, nrhs, part, nb, st0, st1, bb, n_active,
                     limit);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int cg_finalize_launch(int nrhs, const ColState* st, const double* bb, double* bnorm2, int* iters, double* relres,
                       int* status, int n_lanczos, double* ab, hipStream_t stream) {
  hipLaunchKernelGGL(cg_finalize_kernel, dim3(cdiv(nrhs, 256)), dim3(256), 0, stream, nrhs, st, bb, bnorm2, iters,
                     relres, status, n_lanczos, ab);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

// Host polling resources, one set per host thread.
struct PollSlots {
  int* flags = nullptr;  // coherent pinned host memory, 2 slots
  hipEvent_t ev[2] = {nullptr, nullptr};
  int device = -1;
};

static int poll_slots(PollSlots*& out) {
  thread_local PollSlots slots;
  int dev = 0;
  GPL_HIP(hipGetDevice(&dev));
  if (slots.flags == nullptr || slots.device != dev) {
    GPL_HIP(hipHostMalloc(reinterpret_cast<void**>(&slots.flags), 2 * sizeof(int), hipHostMallocCoherent));
    GPL_HIP(hipEventCreateWithFlags(&slots.ev[0], hipEventDisableTiming));
    GPL_HIP(hipEventCreateWithFlags(&slots.ev[1], hipEventDisableTiming));
    slots.device = dev;
  }
  out = &slots;
  return GPL_OK;
}

static int check_problem(const gpl_problem* prob, Taps& taps, bool windowed_ok = false) {
  GPL_REQUIRE(prob != nullptr, "problem is NULL");
  const gpl_grid* g = &prob->grid;
  GPL_REQUIRE(g->n >= 1 && g->ss >= 1 && g->pix_scale > 0, "bad grid");
  GPL_REQUIRE(prob->px && prob->py, "problem points are NULL");
  GPL_REQUIRE(prob->noise_sigma >= 0 && std::isfinite(prob->noise_sigma), "noise_sigma must be >= 0");
  GPL_TRY(windowed_ok ? check_kernel_any(&prob->kernel) : check_kernel(&prob->kernel));
  GPL_TRY(make_taps(g, &prob->psf, taps));
  return GPL_OK;
}

// One application of A to the columns of P: AP = B K B^T P + sigma^2 P, with
// p.Ap partials when `pap` is given.
static int apply_A_into(const gpl_problem* prob, const Taps& taps, const MvmCtx& mv, int nrhs, const float* P,
                        int ldp, float* T1, float* T2, int ldf, float* AP, int ldap, double* pap, CgGate gate,
                        hipStream_t stream) {
  const int n = prob->grid.n, ss = prob->grid.ss;
  const float s2 = (float)(prob->noise_sigma * prob->noise_sigma);
  GPL_TRY(psf_adjoint_launch(n, ss, taps, nrhs, P, ldp, T1, ldf, 1.f, 0.f, gate, stream));
  GPL_TRY(mvm_run(mv, nrhs, T1, ldf, T2, ldf, 0.f, gate, stream));
  GPL_TRY(psf_forward_launch(n, ss, taps, nrhs, T2, ldf, AP, ldap, 1.f, 0.f, P, ldp, s2, pap ? P : nullptr, ldp, pap,
                             gate, stream));
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" size_t gpl_apply_A_workspace(const gpl_problem* prob, int nrhs, int prec) {
  if (prob == nullptr || nrhs <= 0) return 0;
  const int N = prob->grid.n * prob->grid.ss * prob->grid.n * prob->grid.ss;
  Sizer s;
  const int ldf = round_up(N, 64);
  s.take<float>((size_t)ldf * nrhs);
  s.take<float>((size_t)ldf * nrhs);
  s.take<char>(mvm_workspace(N, nrhs, prec));
  return s.used;
}

extern "C" int gpl_apply_A(const gpl_problem* prob, int nrhs, const float* X, int ldx, float* Y, int ldy, int prec,
                           void* ws, size_t ws_bytes, hipStream_t stream) {
  Taps taps;
  GPL_TRY(check_problem(prob, taps, true));
  GPL_REQUIRE(nrhs >= 0 && nrhs <= 65535, "nrhs out of range");
  if (nrhs == 0) return GPL_OK;
  const int npix = prob->grid.n * prob->grid.n, N = npix * prob->grid.ss * prob->grid.ss;
  GPL_REQUIRE(X && Y && X != Y, "X/Y NULL or aliased");
  GPL_REQUIRE(ldx >= npix && ldy >= npix, "ldx/ldy must be >= n*n");
  GPL_TRY(check_ws(ws, ws_bytes, gpl_apply_A_workspace(prob, nrhs, prec)));
  Carver c(ws, ws_bytes);
  const int ldf = round_up(N, 64);
  float* T1 = c.take<float>((size_t)ldf * nrhs);
  float* T2 = c.take<float>((size_t)ldf * nrhs);
  const size_t mb = mvm_workspace(N, nrhs, prec);
  char* mws = c.take<char>(mb);
  if (!c.ok()) return check_ws(nullptr, 0, 1);
  if (prob->kernel.kind == 1) {  // windowed kernel: B^T, the Gaussian product with pixel shapes, B
    if (prec != GPL_PREC_FP32) {
      set_error("the windowed kernel (kind 1) runs in the FP32 form only");
      return GPL_EUNSUPPORTED;
    }
    const int n = prob->grid.n, ss = prob->grid.ss;
    const float s2 = (float)(prob->noise_sigma * prob->noise_sigma);
    GPL_TRY(psf_adjoint_launch(n, ss, taps, nrhs, X, ldx, T1, ldf, 1.f, 0.f, CgGate{}, stream));
    GPL_TRY(windowed_mvm(&prob->kernel, &prob->grid, N, prob->px, prob->py, nrhs, T1, ldf, T2, ldf, 0.f, mws, mb,
                         stream));
    return psf_forward_launch(n, ss, taps, nrhs, T2, ldf, Y, ldy, 1.f, 0.f, X, ldx, s2, nullptr, 0, nullptr,
                              CgGate{}, stream);
  }
  MvmCtx mv;
  GPL_TRY(mvm_prepare(mv, prob->kernel.lengthscale, prob->kernel.amplitude, N, prob->px, prob->py, &prob->grid, nrhs,
                      prec, mws, mb, stream));
  return apply_A_into(prob, taps, mv, nrhs, X, ldx, T1, T2, ldf, Y, ldy, nullptr, CgGate{}, stream);
}

extern "C" size_t gpl_cg_solve_workspace(const gpl_problem* prob, int nrhs, int prec) {
  if (prob == nullptr || nrhs <= 0 || prob->grid.n <= 0 || prob->grid.ss <= 0) return 0;
  const int npix = prob->grid.n * prob->grid.n, N = npix * prob->grid.ss * prob->grid.ss;
  Sizer s;
  carve_cg(s, npix, N, nrhs, prec, nullptr, nullptr, prob->grid.ss, prob->grid.n);
  return s.used;
}

extern "C" int gpl_cg_solve(const gpl_problem* prob, int nrhs, const float* Bm, int ldb, float* X, int ldx,
                            double tol, int max_iter, int fixed_iters, int n_lanczos, double* lanczos_ab,
                            double* bnorm2, int* iters, double* relres, double* true_relres, int* status, int prec,
                            int check_every, void* ws, size_t ws_bytes, hipStream_t stream) {
  Taps taps;
  GPL_TRY(check_problem(prob, taps));
  GPL_REQUIRE(nrhs >= 1 && nrhs <= 65535, "nrhs=%d out of range", nrhs);
  GPL_REQUIRE(prec == GPL_PREC_FP32 || prec == GPL_PREC_F16X3, "unknown precision %d", prec);
  const int n = prob->grid.n, ss = prob->grid.ss, npix = n * n, N = npix * ss * ss;
  GPL_REQUIRE(Bm && X, "Bm/X are NULL");
  GPL_REQUIRE(ldb >= npix && ldx >= npix, "ldb/ldx must be >= n*n");
  GPL_REQUIRE(tol >= 0 && max_iter >= 0 && fixed_iters >= 0 && n_lanczos >= 0, "negative tol/iteration counts");
  GPL_REQUIRE(n_lanczos == 0 || lanczos_ab != nullptr, "lanczos_ab is NULL");
  GPL_REQUIRE(check_every >= 0, "check_every must be >= 0");
  GPL_TRY(check_ws(ws, ws_bytes, gpl_cg_solve_workspace(prob, nrhs, prec)));
  Carver cv(ws, ws_bytes);
  CgBuffers b;
  carve_cg(cv, npix, N, nrhs, prec, &b, nullptr, ss, n);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);
  PollSlots* poll = nullptr;
  if (check_every > 0) GPL_TRY(poll_slots(poll));
  MvmCtx mv;  // the points stay fixed for the whole solve: one tile plan
  GPL_TRY(mvm_prepare(mv, prob->kernel.lengthscale, prob->kernel.amplitude, N, prob->px, prob->py, &prob->grid, nrhs,
                      prec, b.mvm_ws, b.mvm_ws_bytes, stream));
  const RhsOut rhs_out{prec, nrhs, mv.bufs.ncp, mv.bufs.Vh, mv.bufs.Vl, mv.bufs.Vp, mv.bufs.inv_scale, b.pmax, b.nb_upd,
                       mv.plan.irank};
  const float sigma2 = (float)(prob->noise_sigma * prob->noise_sigma);

  const int nb = b.nb_upd;
  const int limit = fixed_iters > 0 ? fixed_iters : max_iter;
  hipLaunchKernelGGL(cg_init_kernel, dim3(nb, nrhs), dim3(256), 0, stream, npix, Bm, ldb, X, ldx, b.R, b.P, b.ldv,
                     b.rr_part, nb, b.pmax);
  GPL_LAUNCH_CHECK();
  hipLaunchKernelGGL(cg_init_state_kernel, dim3(1), dim3(256), 0, stream, nrhs, b.rr_part, nb, b.st[0], b.st[1], b.bb,
                     b.n_active, limit);
  GPL_LAUNCH_CHECK();

  // check_every = 0: every iteration up to the limit is enqueued at once, and
  // those after the last column has stopped exit at their first load.
  const int chunk = check_every > 0 ? check_every : std::max(limit, 1);
  const int nchunks = cdiv(limit, chunk);
  int last_end = 0;  // one past the last enqueued iteration
  auto enqueue_chunk = [&](int k) -> int {
    const int end = std::min(limit, (k + 1) * chunk);
    for (int it = k * chunk; it < end; ++it) {
      const int p = it & 1;
      CgGate gate;
      gate.n_active = b.n_active + p;
      // AP = B K B^T P + sigma^2 P with p.Ap partials; B^T P goes straight into
      // the product's RHS buffers
      GPL_TRY(psf_adjoint_rhs_launch(n, ss, taps, nrhs, b.P, b.ldv, rhs_out, gate, stream));
      GPL_TRY(mvm_run_prepared(mv, nrhs, b.T2, b.ldf, 0.f, gate, stream));
      GPL_TRY(psf_forward_launch(n, ss, taps, nrhs, b.T2, b.ldf, b.AP, b.ldv, 1.f, 0.f, b.P, b.ldv, sigma2, b.P, b.ldv,
                                 b.pap_part, gate, stream));
      hipLaunchKernelGGL(cg_update1_kernel, dim3(nb, nrhs), dim3(256), 0, stream, npix, X, ldx, b.R, b.P, b.AP, b.ldv,
                         b.pap_part, b.ntiles, b.rr_part, nb, b.st[p], b.st[1 - p], b.n_active + p,
                         b.n_active + (1 - p));
      GPL_LAUNCH_CHECK();
      hipLaunchKernelGGL(cg_update2_kernel, dim3(nb, nrhs), dim3(256), 0, stream, npix, b.R, b.P, b.ldv, b.rr_part,
                         nb, b.st[p], b.st[1 - p], b.bb, b.n_active + p, b.n_active + (1 - p), tol, max_iter,
                         fixed_iters, n_lanczos, lanczos_ab, b.pmax);
      GPL_LAUNCH_CHECK();
    }
    last_end = end;
    if (!poll) return GPL_OK;
    hipLaunchKernelGGL(cg_snapshot_kernel, dim3(1), dim3(64), 0, stream, b.n_active + (end & 1),
                       poll->flags + (k & 1));
    GPL_LAUNCH_CHECK();
    GPL_HIP(hipEventRecord(poll->ev[k & 1], stream));
    return GPL_OK;
  };

  if (nchunks > 0 && !poll) {
    GPL_TRY(enqueue_chunk(0));
  } else if (nchunks > 0) {
    GPL_TRY(enqueue_chunk(0));
    for (int k = 0; k < nchunks; ++k) {
      if (k + 1 < nchunks) GPL_TRY(enqueue_chunk(k + 1));
      GPL_HIP(hipEventSynchronize(poll->ev[k & 1]));
      if (poll->flags[k & 1] == 0) break;  // later iterations only carry the state forward
    }
  }
  const int final_parity = last_end & 1;
  hipLaunchKernelGGL(cg_finalize_kernel, dim3(cdiv(nrhs, 256)), dim3(256), 0, stream, nrhs, b.st[final_parity], b.bb,
                     bnorm2, iters, relres, status, n_lanczos, lanczos_ab);
  GPL_LAUNCH_CHECK();
  if (true_relres) {
    // |b - A x| / |b| of the returned iterate: one more application of A, to X
    // itself (the recursive residual R drifts from it in finite precision)
    hipLaunchKernelGGL(cg_absmax_kernel, dim3(nb, nrhs), dim3(256), 0, stream, npix, X, ldx, b.pmax, nb);
    GPL_LAUNCH_CHECK();
    GPL_TRY(psf_adjoint_rhs_launch(n, ss, taps, nrhs, X, ldx, rhs_out, CgGate{}, stream));
    GPL_TRY(mvm_run_prepared(mv, nrhs, b.T2, b.ldf, 0.f, CgGate{}, stream));
    GPL_TRY(psf_forward_launch(n, ss, taps, nrhs, b.T2, b.ldf, b.AP, b.ldv, 1.f, 0.f, X, ldx, sigma2, nullptr, 0,
                               nullptr, CgGate{}, stream));
    hipLaunchKernelGGL(cg_true_residual_kernel, dim3(nb, nrhs), dim3(256), 0, stream, npix, Bm, ldb, b.AP, b.ldv,
                       b.rr_part, nb);
    GPL_LAUNCH_CHECK();
    hipLaunchKernelGGL(cg_true_residual_fold_kernel, dim3(cdiv(nrhs, 256)), dim3(256), 0, stream, nrhs, b.rr_part,
                       nb, b.bb, true_relres);
    GPL_LAUNCH_CHECK();
  }
  return GPL_OK;
}
