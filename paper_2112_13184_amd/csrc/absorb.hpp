// Fused single-layer absorption of a site into an edge-corner product.
#pragma once

#include "common.hpp"

namespace ctm {

// True if the fused kernel handles these dimensions (D^4 d blocks up to
// D = 8, d = 2, and a double-layer network).
bool absorb_fused_fits(int DK, int DB, int d);

// G[(cn, r, r'), (cp, dd, d')] (transposed: G[(cp, dd, d'), (cn, r, r')]) =
//   sum X[(cp, l, l'), (cn, u, u')] Ak[l, u, r, dd, p] Ab[l', u', r', d', p]
// for n x n row-major X and G, n = chi DK DB; Ak, Ab row-major [l][u][r][d][p].
// amax (device, nullable): receives max(*amax, largest |G|) as FP32 bits.
void absorb_fused(hipStream_t st, const double* X, const double* Ak, const double* Ab, double* G, int chi,
                  int DK, int DB, int d, bool transposed, unsigned* amax = nullptr);

// The same for `batch` problems of one shape in one launch, problem b taking
// X + xo[b], Ak + ako[b], Ab + abo[b] and G + go[b] (device arrays of element
// offsets; with batch = 1 they may be null).  amaxp (device table of
// pointers, nullable): problem b's largest |G| into *amaxp[b] (FP32 bits,
// atomic max); amax1: the same for a single problem.
void absorb_fused_batched(hipStream_t st, const double* X, const double* Ak, const double* Ab, double* G,
                          const long* xo, const long* ako, const long* abo, const long* go, int batch, int chi,
                          int DK, int DB, int d, bool transposed, unsigned* const* amaxp = nullptr,
                          unsigned* amax1 = nullptr);

}  // namespace ctm
