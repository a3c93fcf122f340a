// Continuous-batching request loop on the device: each admitted reconstruction
// (a "slot") keeps its points, CG vectors, CG state and Lanczos coefficients in
// its own workspace; one CG iteration of every active slot is a fixed sequence
// of grouped launches (PSF adjoint, kernel product, PSF + sigma^2, updates),
// each a single launch whose workgroups decode their (slot, tile) from offsets
// passed by value. Every slot keeps its own tile plan and reduction order, so
// its results do not depend on which other slots share the launches.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "internal.hpp"
#include "mvm_mfma.hpp"

namespace gpl {

static_assert(sizeof(ServeSlotDev) <= sizeof(((gpl_serve_slot*)nullptr)->opaque), "slot descriptor too large");

static const ServeSlotDev& host_desc(const gpl_serve_slot* s) {
  return *reinterpret_cast<const ServeSlotDev*>(s->opaque);
}

// Buffers of one slot, in carving order. The descriptor sits first.
struct SlotBufs {
  ServeSlotDev* desc;
  float *px, *py, *mu, *rhs, *X, *R, *P, *AP, *T2, *w;
  TilePlan plan;
  unsigned* pmax;
  float* inv_scale;
  _Float16 *Vh, *Vl;
  float *Vp, *part;
  ColState *st0, *st1;
  double *bb, *pap, *rr, *ab, *bnorm2, *contrib, *scal, *lz_ws;
  int* n_active;
  char* mv_ws;
  size_t mv_bytes, lz_bytes;
};

template <class Cv>
static void carve_slot(Cv& cv, int n, int ss, int nrhs, int n_lanczos, int prec, SlotBufs* b) {
  const int npix = n * n, N = npix * ss * ss;
  const int ldv = round_up(npix, 64), ldf = round_up(N, 64);
  const int nrt = cdiv(N, kRowTile), ldh = nrt * kRowTile, ncp = cdiv(nrhs, 16) * 16;
  const bool f16 = prec == GPL_PREC_F16X3;
  const int ntiles = psf_forward_tiles(n, ss), nb = cg_blocks(npix);
  SlotBufs x;
  x.desc = cv.template take<ServeSlotDev>(1);
  x.px = cv.template take<float>(N);
  x.py = cv.template take<float>(N);
  x.mu = cv.template take<float>(N);
  x.rhs = cv.template take<float>((size_t)ldv * nrhs);
  x.X = cv.template take<float>((size_t)ldv * nrhs);
  x.R = cv.template take<float>((size_t)ldv * nrhs);
  x.P = cv.template take<float>((size_t)ldv * nrhs);
  x.AP = cv.template take<float>((size_t)ldv * nrhs);
  x.T2 = cv.template take<float>((size_t)ldf * nrhs);
  x.w = cv.template take<float>(N);
  plan_carve(cv, N, x.plan);
  x.pmax = cv.template take<unsigned>((size_t)nrhs * nb);
  x.inv_scale = cv.template take<float>(ncp);
  x.Vh = cv.template take<_Float16>(f16 ? (size_t)ncp * ldh : 1);
  x.Vl = cv.template take<_Float16>(f16 ? (size_t)ncp * ldh : 1);
  x.Vp = cv.template take<float>(f16 ? 1 : (size_t)ncp * ldh);
  x.part = cv.template take<float>((size_t)plan_slots(N) * nrhs * kRowTile);
  x.st0 = cv.template take<ColState>(nrhs);
  x.st1 = cv.template take<ColState>(nrhs);
  x.bb = cv.template take<double>(nrhs);
  x.n_active = cv.template take<int>(2);
  x.pap = cv.template take<double>((size_t)ntiles * nrhs);
  x.rr = cv.template take<double>((size_t)nb * nrhs);
  x.ab = cv.template take<double>((size_t)nrhs * std::max(n_lanczos, 1) * 2);
  x.bnorm2 = cv.template take<double>(nrhs);
  x.contrib = cv.template take<double>(nrhs);
  x.scal = cv.template take<double>(8);
  x.lz_bytes = gpl_lanczos_logdet_workspace(std::max(nrhs - 1, 1), std::max(n_lanczos, 1));
  x.lz_ws = reinterpret_cast<double*>(cv.template take<char>(x.lz_bytes));
  x.mv_bytes = mvm_workspace(N, 1, GPL_PREC_FP32);
  x.mv_ws = cv.template take<char>(x.mv_bytes);
  if (b) *b = x;
}

__global__ void fill_nan_kernel(double* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = __builtin_nan("");
}

__global__ void write_desc_kernel(ServeSlotDev d, ServeSlotDev* out) {
  if (threadIdx.x == 0) *out = d;
}

__global__ void serve_snapshot_kernel(SlotBatch B, int p, int* host_active) {
  const int s = threadIdx.x;
  if (s < B.nslots) {
    *(volatile int*)(host_active + s) = B.slot[s]->n_active[p];
    __threadfence_system();
  }
}

static int check_slots(gpl_serve_slot* const* slots, int nslots) {
  GPL_REQUIRE(nslots >= 0 && nslots <= kMaxServeSlots, "nslots=%d must be in [0, %d]", nslots, kMaxServeSlots);
  for (int s = 0; s < nslots; ++s)
    GPL_REQUIRE(slots[s] != nullptr && slots[s]->dev != nullptr, "slot %d is not initialised", s);
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" size_t gpl_serve_slot_workspace(const gpl_grid* grid, int nrhs, int n_lanczos, int prec) {
  if (grid == nullptr || grid->n < 1 || grid->ss < 1 || nrhs < 1 || nrhs > 32) return 0;
  Sizer s;
  carve_slot(s, grid->n, grid->ss, nrhs, n_lanczos, prec, nullptr);
  return s.used;
}

extern "C" int gpl_serve_slot_init(gpl_serve_slot* slot, const gpl_problem* prob, const gpl_lens* lens,
                                   const gpl_source* src, const float* d, const float* probes, int ldz, int nrhs,
                                   double tol, int max_iter, int n_lanczos, int prec, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
  GPL_REQUIRE(slot && prob && lens && src && d, "NULL argument");
  GPL_REQUIRE(nrhs >= 1 && nrhs <= 32, "nrhs=%d must be in [1, 32] for a serving slot", nrhs);
  GPL_REQUIRE(nrhs == 1 || probes != nullptr, "probes are NULL");
  GPL_REQUIRE(prec == GPL_PREC_FP32 || prec == GPL_PREC_F16X3, "unknown precision %d", prec);
  GPL_REQUIRE(tol >= 0 && max_iter >= 1 && n_lanczos >= 0, "bad tol / max_iter / n_lanczos");
  GPL_TRY(check_kernel(&prob->kernel));
  const gpl_grid* g = &prob->grid;
  Taps taps;
  GPL_TRY(make_taps(g, &prob->psf, taps));
  const int n = g->n, ss = g->ss, npix = n * n, N = npix * ss * ss;
  GPL_REQUIRE(n >= 1 && ss >= 1 && ss <= 32 && (long)n * ss < 32768, "grid n=%d ss=%d out of range", n, ss);
  GPL_REQUIRE(nrhs == 1 || ldz >= npix, "ldz must be >= n*n");
  GPL_TRY(check_ws(ws, ws_bytes, gpl_serve_slot_workspace(g, nrhs, n_lanczos, prec)));
  Carver cv(ws, ws_bytes);
  SlotBufs b;
  carve_slot(cv, n, ss, nrhs, n_lanczos, prec, &b);
  if (!cv.ok()) return check_ws(nullptr, 0, 1);

  ServeSlotDev D;
  std::memset(&D, 0, sizeof(D));
  D.n = n;
  D.ss = ss;
  D.npix = npix;
  D.N = N;
  D.nrhs = nrhs;
  D.prec = prec;
  D.taps = taps;
  D.sigma2 = (float)(prob->noise_sigma * prob->noise_sigma);
  D.s2 = (float)kernel_scale2(prob->kernel.lengthscale);
  D.amp2 = (float)(prob->kernel.amplitude * prob->kernel.amplitude);
  D.px = b.px;
  D.py = b.py;
  D.X = b.X;
  D.R = b.R;
  D.P = b.P;
  D.AP = b.AP;
  D.T2 = b.T2;
  D.ldv = round_up(npix, 64);
  D.ldf = round_up(N, 64);
  D.plan = b.plan;
  D.pmax = b.pmax;
  D.inv_scale = b.inv_scale;
  D.Vh = b.Vh;
  D.Vl = b.Vl;
  D.Vp = b.Vp;
  D.part = b.part;
  D.ldh = b.plan.npad;
  D.ncp = cdiv(nrhs, 16) * 16;
  D.st[0] = b.st0;
  D.st[1] = b.st1;
  D.bb = b.bb;
  D.n_active = b.n_active;
  D.pap_part = b.pap;
  D.rr_part = b.rr;
  D.ntiles_fwd = psf_forward_tiles(n, ss);
  D.ntiles_adj = psf_adjoint_tiles(n, ss);
  D.nb_upd = cg_blocks(npix);
  D.ab = b.ab;
  D.n_lanczos = n_lanczos;
  D.max_iter = max_iter;
  D.tol = tol;
  D.ell = prob->kernel.lengthscale;
  D.amp = prob->kernel.amplitude;
  D.sigma = prob->noise_sigma;

  hipLaunchKernelGGL(write_desc_kernel, dim3(1), dim3(64), 0, stream, D, b.desc);
  GPL_LAUNCH_CHECK();
  // the grouped PSF adjoint writes only the slot's fine points and columns:
  // the padding of the RHS buffers stays zero
  const ProdBufs pb{nullptr, b.inv_scale, b.Vh, b.Vl, b.Vp, b.part, D.ldh, D.ncp};
  GPL_TRY(mfma_zero_rhs(pb, prec, stream));
  GPL_TRY(gpl_lens_raytrace(g, lens, b.px, b.py, stream));
  TilePlan plan = b.plan;  // same buffers as the descriptor's copy
  GPL_TRY(plan_build(plan, N, b.px, b.py, g, D.s2, plan_threshold(prec), plan_lo_threshold(prec), stream));
  GPL_TRY(gpl_sersic_eval(src, N, b.px, b.py, b.mu, stream));
  GPL_HIP(hipMemcpyAsync(b.rhs, d, sizeof(float) * npix, hipMemcpyDeviceToDevice, stream));
  if (nrhs > 1)
    GPL_HIP(hipMemcpy2DAsync(b.rhs + D.ldv, sizeof(float) * D.ldv, probes, sizeof(float) * ldz, sizeof(float) * npix,
                             nrhs - 1, hipMemcpyDeviceToDevice, stream));
  // residual r = d - B mu in column 0
  GPL_TRY(psf_forward_launch(n, ss, taps, 1, b.mu, N, b.rhs, D.ldv, -1.f, 1.f, nullptr, 0, 0.f, nullptr, 0, nullptr,
                             CgGate{}, stream));
  GPL_TRY(cg_init_launch(npix, nrhs, b.rhs, D.ldv, b.X, D.ldv, b.R, b.P, D.ldv, b.rr, b.st0, b.st1, b.bb, b.n_active,
                         max_iter, b.pmax, stream));
  std::memcpy(slot->opaque, &D, sizeof(D));
  slot->dev = b.desc;
  slot->ws = ws;
  slot->N = N;
  slot->npix = npix;
  slot->nrhs = nrhs;
  return GPL_OK;
}

extern "C" int gpl_serve_step(gpl_serve_slot* const* slots, int nslots, int iters, long iter0, hipStream_t stream) {
  GPL_TRY(check_slots(slots, nslots));
  GPL_REQUIRE(iters >= 0 && iter0 >= 0, "negative iteration count");
  if (nslots == 0) return GPL_OK;
  const ServeSlotDev* h[kMaxServeSlots];
  const ServeSlotDev* dv[kMaxServeSlots];
  for (int s = 0; s < nslots; ++s) {
    h[s] = &host_desc(slots[s]);
    dv[s] = static_cast<const ServeSlotDev*>(slots[s]->dev);
  }
  for (int k = 0; k < iters; ++k) {
    const int p = (int)((iter0 + k) & 1);
    GPL_TRY(psf_adjoint_grouped(h, dv, nslots, p, stream));
    GPL_TRY(mvm_grouped(h, dv, nslots, p, stream));
    GPL_TRY(psf_forward_grouped(h, dv, nslots, p, stream));
    GPL_TRY(cg_update_grouped(h, dv, nslots, p, stream));
  }
  return GPL_OK;
}

extern "C" int gpl_serve_snapshot(gpl_serve_slot* const* slots, int nslots, long iter, int* host_active,
                                  hipStream_t stream) {
  GPL_TRY(check_slots(slots, nslots));
  GPL_REQUIRE(host_active != nullptr, "host_active is NULL");
  if (nslots == 0) return GPL_OK;
  SlotBatch B;
  B.nslots = nslots;
  for (int s = 0; s < nslots; ++s) B.slot[s] = static_cast<const ServeSlotDev*>(slots[s]->dev);
  hipLaunchKernelGGL(serve_snapshot_kernel, dim3(1), dim3(64), 0, stream, B, (int)(iter & 1), host_active);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" int gpl_serve_slot_finish(gpl_serve_slot* slot, long iter, double logdet_scale, double* out, int* iters,
                                     double* relres, int* status, float* fhat, float* image, hipStream_t stream) {
  GPL_REQUIRE(slot && slot->dev && out && iters && relres && status, "NULL argument");
  const ServeSlotDev& D = host_desc(slot);
  Carver cv(slot->ws, (size_t)-1);
  SlotBufs b;
  carve_slot(cv, D.n, D.ss, D.nrhs, D.n_lanczos, D.prec, &b);
  const int p = (int)(iter & 1);
  GPL_TRY(cg_finalize_launch(D.nrhs, p ? b.st1 : b.st0, b.bb, b.bnorm2, iters, relres, status, D.n_lanczos, b.ab,
                             stream));
  double* logdet = b.scal + 3;
  double* stderr_ = b.scal + 4;
  const int m = D.nrhs - 1;
  if (m > 0 && D.n_lanczos > 0) {
    GPL_TRY(gpl_lanczos_logdet(m, D.n_lanczos, b.ab + (size_t)D.n_lanczos * 2, iters + 1, b.bnorm2 + 1, logdet_scale,
                               nullptr, b.contrib, logdet, stderr_, b.lz_ws, b.lz_bytes, stream));
  } else {
    hipLaunchKernelGGL(fill_nan_kernel, dim3(1), dim3(64), 0, stream, logdet, 2);  // no log-determinant requested
    GPL_LAUNCH_CHECK();
  }
  GPL_TRY(gpl_evidence_scalars(D.npix, D.N, b.rhs, b.X, logdet, D.amp, D.sigma, b.scal, stream));
  GPL_HIP(hipMemcpyAsync(out, b.scal, 5 * sizeof(double), hipMemcpyDeviceToDevice, stream));
  if (fhat) {
    // posterior mean mu + K B^T u and the predicted image B fhat
    GPL_TRY(psf_adjoint_launch(D.n, D.ss, D.taps, 1, b.X, D.ldv, b.w, D.N, 1.f, 0.f, CgGate{}, stream));
    GPL_HIP(hipMemcpyAsync(fhat, b.mu, sizeof(float) * D.N, hipMemcpyDeviceToDevice, stream));
    gpl_grid grid{D.n, D.ss, 0.0, 0.0, 0.0};  // ordering only: the points are this grid's fine pixels
    GPL_TRY(mvm_launch(D.ell, D.amp, D.N, D.px, D.py, &grid, 1, b.w, D.N, fhat, D.N, 1.f, GPL_PREC_FP32, b.mv_ws,
                       b.mv_bytes, CgGate{}, stream));
    if (image)
      GPL_TRY(psf_forward_launch(D.n, D.ss, D.taps, 1, fhat, D.N, image, D.npix, 1.f, 0.f, nullptr, 0, 0.f, nullptr, 0,
                                 nullptr, CgGate{}, stream));
  }
  return GPL_OK;
}
