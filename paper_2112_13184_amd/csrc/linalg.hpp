// FP64 dense factorisations used by the projector computation.
#pragma once

#include "common.hpp"

namespace ctm {

struct Linalg;   // opaque: owns the solver handle and its scratch

Linalg* linalg_create(hipStream_t st);
void linalg_destroy(Linalg* la);

// Y (n x k, column-major, ld = n, n >= k) <- orthonormal basis of its range
// (Householder QR).
void la_orth(Linalg* la, double* Y, int n, int k);

// Z (n x k, column-major, n >= k) <- Q, and R (k x k, column-major) <- the
// upper-triangular factor, with Z = Q R.
void la_qr(Linalg* la, double* Z, int n, int k, double* R);

// A (k x k, column-major) = U diag(S) V^T; writes U and VT (both k x k,
// column-major; VT holds V^T).  A is destroyed.  S descending.
void la_svd(Linalg* la, double* A, int k, double* S, double* U, double* VT);

// A (n x n symmetric, column-major; the lower triangle is read) <- its
// eigenvectors (columns), W <- the eigenvalues, ascending.
void la_syev(Linalg* la, double* A, int n, double* W);

// Singular values (descending) of `batch` m x m column-major matrices stored
// back to back; A is destroyed.  S: batch x m.
void la_singular_values_batched(Linalg* la, double* A, int m, int batch, double* S);

}  // namespace ctm
