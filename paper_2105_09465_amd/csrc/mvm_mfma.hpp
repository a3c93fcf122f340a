// Kernel-matrix product over the pairs of a tile plan on MFMA: the precision
// form (FP32 exp tiles split into FP16 hi/lo, FP16 hi/lo RHS, FP32 accumulation)
// and the FP32 form.
#pragma once

#include "internal.hpp"
#include "tileplan.hpp"

namespace gpl {

// Scratch bytes of one product of n points and nrhs columns (plan excluded).
size_t mfma_workspace(int n, int nrhs, int prec);
// Skip threshold of the plan for a precision form.
float plan_threshold(int prec);
// Y = amp2 K V + beta Y over the plan P (points P.n, caller order of V and Y).
int mfma_launch(const TilePlan& P, int prec, float s2, float amp2, int nrhs, const float* V, int ldv, float* Y,
                int ldy, float beta, void* ws, size_t ws_bytes, CgGate gate, hipStream_t stream);

}  // namespace gpl
