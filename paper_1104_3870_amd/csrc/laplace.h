// Batched Laplacian / Chebyshev launchers shared by the eigensolver.
#pragma once

#include "laph_impl.h"

// out = alpha Lap(in) + beta in + gamma prev on every slice; vectors of slice t start at
// ptr + t * stride (complex elements); skip[t] != 0 leaves slice t untouched (may be null)
void lap_fused(laph_ctx *c, const double2 *us, const double2 *in, long in_stride, const double2 *prev,
               long prev_stride, double2 *out, long out_stride, double alpha, double beta, double gamma,
               const int *skip);

// out = T_order(B) in with B = 1 + 2/(lamL - lamC) (Lap + lamC); w0, w1 scratch
void cheb_apply(laph_ctx *c, const double2 *us, const double2 *in, long in_stride, double2 *out, long out_stride,
                double2 *w0, double2 *w1, long w_stride, double lamL, double lamC, int order, const int *skip);
