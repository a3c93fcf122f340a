// Internal interfaces between the observation operator, the kernel product and
// the CG driver.
#pragma once

#include "common.hpp"

namespace gpl {

struct Taps {
  int r;
  float w[2 * GPL_PSF_MAX_RADIUS + 1];
};

// Early-exit gate used inside the CG loop: a kernel returns at once when no
// column is active, or when its own column is not.
struct CgGate {
  const int* n_active = nullptr;   // device scalar
  const int* col_active = nullptr; // device [nrhs], stride `stride` ints
  int stride = 1;
  __device__ bool skip(int c) const {
    if (n_active && *n_active == 0) return true;
    if (col_active && col_active[c * stride] == 0) return true;
    return false;
  }
  __device__ bool skip_all() const { return n_active && *n_active == 0; }
};

int make_taps(const gpl_grid* g, const gpl_psf* psf, Taps& t);
int psf_forward_tiles(int n, int ss);
int psf_forward_launch(int n, int ss, const Taps& taps, int nrhs, const float* in, int ld_in, float* out, int ld_out,
                       float alpha, float beta, const float* extra, int ld_extra, float gamma, const float* dotv,
                       int ld_dotv, double* partial, CgGate gate, hipStream_t stream);
int psf_adjoint_launch(int n, int ss, const Taps& taps, int nrhs, const float* in, int ld_in, float* out, int ld_out,
                       float alpha, float beta, CgGate gate, hipStream_t stream);

// Kernel product Y = K V + beta Y (internal form with the CG gate).
size_t mvm_workspace(int n, int nrhs, int prec);
int mvm_launch(double lengthscale, double amplitude, int n, const float* px, const float* py, int nrhs, const float* V,
               int ldv, float* Y, int ldy, float beta, int prec, void* ws, size_t ws_bytes, CgGate gate,
               hipStream_t stream);

int check_kernel(const gpl_kernel* k);

}  // namespace gpl
