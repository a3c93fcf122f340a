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
float plan_threshold(int prec);     // skip threshold on s2 g^2 of the form
float plan_lo_threshold(int prec);  // threshold of the lo masks (the skip threshold in the FP32 form)
// Carve the product buffers from a workspace of mfma_workspace bytes.
int mfma_carve(const TilePlan& P, int prec, int nrhs, void* ws, size_t ws_bytes, ProdBufs& b);
// Zero the RHS buffers (padding rows and columns must stay zero).
int mfma_zero_rhs(const ProdBufs& b, int prec, hipStream_t stream);
// RHS block V (caller order) into the product buffers (sorted order, split or packed).
int mfma_prep_rhs(const TilePlan& P, const ProdBufs& b, int prec, int nrhs, const float* V, int ldv, CgGate gate,
                  hipStream_t stream);
// Y = amp2 K V + beta Y (caller order) from the prepared RHS buffers.
int mfma_product(const TilePlan& P, const ProdBufs& b, int prec, float s2, float amp2, int nrhs, float* Y, int ldy,
                 float beta, CgGate gate, hipStream_t stream);

}  // namespace gpl
