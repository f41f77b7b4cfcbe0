// Fused single-layer absorption of a site into an edge-corner product.
#pragma once

#include "common.hpp"

namespace ctm {

// True if the fused kernel handles these dimensions (D^4 d blocks up to
// D = 6, d = 2, and a double-layer network).
bool absorb_fused_fits(int DK, int DB, int d);

// G[(cn, r, r'), (cp, dd, d')] (transposed: G[(cp, dd, d'), (cn, r, r')]) =
//   sum X[(cp, l, l'), (cn, u, u')] Ak[l, u, r, dd, p] Ab[l', u', r', d', p]
// for n x n row-major X and G, n = chi DK DB; Ak, Ab row-major [l][u][r][d][p].
void absorb_fused(hipStream_t st, const double* X, const double* Ak, const double* Ab, double* G, int chi,
                  int DK, int DB, int d, bool transposed);

// The same for `batch` problems of one shape in one launch, problem b taking
// Xp[b], Akp[b], Abp[b] and Gp[b] (device arrays of device pointers; with
// batch = 1 they may be null and X, Ak, Ab, G are used).
void absorb_fused_batched(hipStream_t st, const double* X, const double* Ak, const double* Ab, double* G,
                          const double* const* Xp, const double* const* Akp, const double* const* Abp,
                          double* const* Gp, int batch, int chi, int DK, int DB, int d, bool transposed);

}  // namespace ctm
