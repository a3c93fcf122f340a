// Precision form of the kernel-matrix product (placeholder until the MFMA path lands).
#include "common.hpp"
#include "mvm_mfma.hpp"

namespace gpl {

size_t mfma_f16x3_workspace(int, int) { return 0; }

int mfma_f16x3_launch(float, float, int, const float*, const float*, int, const float*, int, float*, int, float,
                      void*, size_t, CgGate, hipStream_t) {
  set_error("precision form not available");
  return GPL_EUNSUPPORTED;
}

}  // namespace gpl
