// Eigenvalues and eigenvectors of small real upper Hessenberg matrices on the
// host: the Ritz values of the Arnoldi iteration behind the transfer-matrix
// spectrum (the matrices are at most a few hundred wide).
#pragma once

#include <complex>
#include <vector>

namespace ctm {

// Eigenvalues of the n x n upper Hessenberg matrix H (row-major, entries
// below the subdiagonal ignored) by the Francis double-shift QR iteration
// (Golub and Van Loan, Matrix Computations, Sec. 7.5) with deflation at
// negligible subdiagonal entries.  Returns false if the iteration did not
// converge within 40 n steps.
bool hessenberg_eigenvalues(std::vector<double> H, int n, std::vector<std::complex<double>>& lam);

// A unit eigenvector of H for the eigenvalue lam (taken from the routine
// above), by two steps of inverse iteration with a complex LU factorisation
// of H - lam I (partial pivoting; an exactly zero pivot is replaced by a tiny
// one).
std::vector<std::complex<double>> hessenberg_eigenvector(const std::vector<double>& H, int n,
                                                        std::complex<double> lam);

}  // namespace ctm
