// Internal interfaces between the observation operator, the kernel product and
// the CG driver.
#pragma once

#include "common.hpp"
#include "tileplan.hpp"

namespace gpl {

// PSF taps on the fine grid and the composite filter of the PSF followed by the
// ss x ss block sum: g[t + r] = sum_{s < ss} w[s - t] for t in [-r, ss - 1 + r]
// (L = 2 r + ss entries; w taken as zero outside [-r, r]).
constexpr int kMaxComposite = 2 * GPL_PSF_MAX_RADIUS + 32;
struct Taps {
  int r, L;
  float w[2 * GPL_PSF_MAX_RADIUS + 1];
  float g[kMaxComposite];
};

// Early-exit gate used inside the CG loop: a kernel returns at once when no
// column is active, or when its own column is not.
struct CgGate {
  const int* n_active = nullptr;   // device scalar
  const int* col_active = nullptr; // device [nrhs], stride `stride` ints
  int stride = 1;
  // products only: when set, a chunk c whose chunk_gen[c] differs from gen has
  // a zero right-hand side in every column and is not evaluated
  const int* chunk_gen = nullptr;
  int gen = 0;
  // both flags are loaded together (one memory round trip, not two)
  __device__ bool skip(int c) const {
    const int na = n_active ? *n_active : 1;
    const int ca = col_active ? col_active[c * stride] : 1;
    return na == 0 || ca == 0;
  }
  __device__ bool skip_all() const { return n_active && *n_active == 0; }
};

struct ColState {
  double rr;     // r.r of the current residual
  double alpha;  // alpha of the step that produced this state
  int active;
  int iters;
  int status;
  int bad;  // set by update1 when p.Ap <= 0 or non-finite
};

// Device-resident descriptor of one request in the serving loop (stored at the
// start of the request's workspace). Every grouped kernel reads its slot's
// sizes and buffers from here.
struct ServeSlotDev {
  int n, ss, npix, N, nrhs, prec;
  Taps taps;
  float sigma2, s2, amp2;
  const float *px, *py;
  float *X, *R, *P, *AP, *T2;
  int ldv, ldf;
  TilePlan plan;  // tile plan of the slot's points
  unsigned* pmax;  // [nrhs][nb_upd] partial max |P| (float bits)
  float* inv_scale;
  _Float16 *Vh, *Vl;  // precision form: RHS block split in sorted order
  float* Vp;          // FP32 form: RHS block in sorted order
  float* part;        // partial rows of the product's work items
  int ldh, ncp;
  ColState* st[2];
  double* bb;
  int* n_active;  // [2]
  double *pap_part, *rr_part;
  int ntiles_fwd, ntiles_adj, nb_upd;
  double* ab;
  int n_lanczos, max_iter;
  double tol;
  double ell, amp, sigma;  // kernel hyperparameters and noise in FP64
};

constexpr int kMaxServeSlots = 64;
// CG vector kernels: each workgroup of 256 threads takes kUpdPer entries per
// thread, entries bx kUpdSpan + e 256 + t (e < kUpdPer), and writes one partial
// (r.r, p.Ap, max |p|) per column.
constexpr int kUpdPer = 4, kUpdSpan = 256 * kUpdPer;
inline int cg_blocks(int npix) { return cdiv(npix, kUpdSpan); }
constexpr int kColmaxBlocks = 32;  // workgroups per column of the column-max pass

// Kernel argument naming the slots of one grouped launch: slot s owns the
// workgroups [off[s], off[s+1]) of the launch.
struct SlotBatch {
  int nslots;
  int off[kMaxServeSlots + 1];
  const ServeSlotDev* slot[kMaxServeSlots];
  __device__ int find(int b) const {
    int s = 0;
    while (s + 1 < nslots && off[s + 1] <= b) ++s;
    return s;
  }
};

int make_taps(const gpl_grid* g, const gpl_psf* psf, Taps& t);
int psf_forward_tiles(int n, int ss);
int psf_forward_launch(int n, int ss, const Taps& taps, int nrhs, const float* in, int ld_in, float* out, int ld_out,
                       float alpha, float beta, const float* extra, int ld_extra, float gamma, const float* dotv,
                       int ld_dotv, double* partial, CgGate gate, hipStream_t stream);
int psf_adjoint_launch(int n, int ss, const Taps& taps, int nrhs, const float* in, int ld_in, float* out, int ld_out,
                       float alpha, float beta, CgGate gate, hipStream_t stream);

// Kernel product Y = K V + beta Y (internal form with the CG gate). A product
// is prepared once per point set (tile plan) and run for any RHS block of at
// most nrhs_max columns. `grid` (nullable) says the points are that grid's fine
// pixels in row-major order.
// Buffers of one product: the RHS block in the plan's sorted order (FP16 hi/lo
// with per-column output scales, or FP32), column-max partials of the RHS, and
// the partial rows of the waves.
struct ProdBufs {
  unsigned* colmax;
  float* inv_scale;
  _Float16 *Vh, *Vl;  // precision form
  float* Vp;          // FP32 form
  float* part;
  int ldh, ncp;
};
struct MvmCtx {
  TilePlan plan;
  ProdBufs bufs;
  int prec, nrhs_max;
  float s2, amp2;
};
size_t mvm_workspace(int n, int nrhs, int prec);
int mvm_prepare(MvmCtx& m, double lengthscale, double amplitude, int n, const float* px, const float* py,
                const gpl_grid* grid, int nrhs, int prec, void* ws, size_t ws_bytes, hipStream_t stream);
int mvm_run(const MvmCtx& m, int nrhs, const float* V, int ldv, float* Y, int ldy, float beta, CgGate gate,
            hipStream_t stream);
// The product from RHS buffers already written (by the fused PSF adjoint).
int mvm_run_prepared(const MvmCtx& m, int nrhs, float* Y, int ldy, float beta, CgGate gate, hipStream_t stream);

// Where the fused PSF adjoint writes B^T P: the product's RHS buffers (fine point
// (fx, fy) at its sorted position in the plan, the FP16 parts of column c at the
// slots hi_slot gives), with per-column scales of the precision form taken from
// partial maxima of |P| (|B^T P| <= max |P| / ss^2).
struct RhsOut {
  int prec;
  int nrhs;  // columns of the product (their FP16 parts are placed by hi_slot)
  int ncp;   // column slots of the buffers (rhs_at layout)
  _Float16 *Vh, *Vl;
  float *Vp, *inv_scale;
  const unsigned* pmax;  // [nrhs][npart] float bits of partial max |P|
  int npart;
  const int* irank;  // fine point (row-major) -> sorted position of the product's plan
};
int psf_adjoint_rhs_launch(int n, int ss, const Taps& taps, int nrhs, const float* P, int ldp, const RhsOut& out,
                           CgGate gate, hipStream_t stream);
int mvm_launch(double lengthscale, double amplitude, int n, const float* px, const float* py, const gpl_grid* grid,
               int nrhs, const float* V, int ldv, float* Y, int ldy, float beta, int prec, void* ws, size_t ws_bytes,
               CgGate gate, hipStream_t stream);

int check_kernel(const gpl_kernel* k);  // RBF only (kind 0)

// Gaussian products with per-point shape covariances (csrc/gauss.hip).
struct GSide {
  const float *x, *y, *z, *w;  // z: SoA zxx[n], zxy[n], zyy[n] (nullable); w nullable
  int n;
};
int gauss_product_launch(const GSide& T, const GSide& S, double base_var, double norm, int nrhs, const float* V,
                         int ldv, float* Y, int ldy, float beta, hipStream_t stream);
int pixel_shapes_launch(int M, const float* px, const float* py, float* z, hipStream_t stream);
int gauss_backward_launch(const GSide& T, const GSide& S, double base_var, double norm, const float* V, const float* U,
                          float* gtx, float* gty, float* gtz, float* gsx, float* gsy, float* gsw, hipStream_t stream);
int pixel_shapes_backward_launch(int M, const float* px, const float* py, const float* gz, float* gab, float* gpx,
                                 float* gpy, hipStream_t stream);
size_t knn_workspace(int n);
int knn_index_launch(int n, const float* qx, const float* qy, int k, float* rho, float* rk, int* nn, void* ws,
                     size_t ws_bytes, hipStream_t stream);
int knn_weight_backward_launch(int n, const float* qx, const float* qy, const float* rk, const int* nn,
                               const float* w, const float* gw, double* gq, float* gpx, float* gpy,
                               hipStream_t stream);
// Ray tracing and its adjoint with the 8 lens parameters in device memory.
size_t raytrace_dev_backward_scratch(int N);
int raytrace_dev_launch(const gpl_grid* grid, const double* lens, float* px, float* py, hipStream_t stream);
int raytrace_dev_backward_launch(const gpl_grid* grid, const double* lens, const float* gpx, const float* gpy,
                                 double* g_lens, double* scratch_partial, hipStream_t stream);
int check_kernel_any(const gpl_kernel* k);  // RBF or windowed (kind 1)
int windowed_mvm(const gpl_kernel* kern, const gpl_grid* grid, int n, const float* px, const float* py, int nrhs,
                 const float* V, int ldv, float* Y, int ldy, float beta, void* ws, size_t ws_bytes,
                 hipStream_t stream);

// Grouped launches of one CG iteration's kernels over the slots of a batch
// (parity p selects the state buffers). Each returns GPL_OK or GPL_EHIP.
int psf_adjoint_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                        hipStream_t stream);
int psf_forward_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                        hipStream_t stream);
int mvm_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                hipStream_t stream);
int cg_update_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                      hipStream_t stream);
int cg_init_launch(int npix, int nrhs, const float* Bm, int ldb, float* X, int ldx, float* R, float* P, int ldv,
                   double* part, ColState* st0, ColState* st1, double* bb, int* n_active, int limit, unsigned* pmax,
                   hipStream_t stream);
int cg_finalize_launch(int nrhs, const ColState* st, const double* bb, double* bnorm2, int* iters, double* relres,
                       int* status, int n_lanczos, double* ab, hipStream_t stream);
int psf_adjoint_tiles(int n, int ss);

}  // namespace gpl
