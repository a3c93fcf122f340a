// Adjoint of the kernel-matrix product (placeholder until the backward lands).
#include "common.hpp"

extern "C" size_t gpl_gp_kernel_mvm_backward_workspace(int, int) { return 0; }

extern "C" int gpl_gp_kernel_mvm_backward(const gpl_kernel*, int, const float*, const float*, int, const float*, int,
                                          const float*, int, const double*, float*, float*, double*, void*, size_t,
                                          hipStream_t) {
  gpl::set_error("kernel-product backward not available");
  return GPL_EUNSUPPORTED;
}
