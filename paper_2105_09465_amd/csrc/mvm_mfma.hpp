// Precision form of the kernel-matrix product: FP32 exp tiles split into FP16
// hi/lo parts and multiplied with the FP16 hi/lo split of the right-hand sides
// on MFMA, FP32 accumulation.
#pragma once

#include "internal.hpp"

namespace gpl {

size_t mfma_f16x3_workspace(int n, int nrhs);
int mfma_f16x3_launch(float s2, float amp2, int n, const float* px, const float* py, int nrhs, const float* V, int ldv,
                      float* Y, int ldy, float beta, void* ws, size_t ws_bytes, CgGate gate, hipStream_t stream);

size_t mfma_f32_workspace(int n, int nrhs);
int mfma_f32_launch(float s2, float amp2, int n, const float* px, const float* py, int nrhs, const float* V, int ldv,
                    float* Y, int ldy, float beta, void* ws, size_t ws_bytes, CgGate gate, hipStream_t stream);

}  // namespace gpl
