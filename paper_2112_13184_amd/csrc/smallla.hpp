// FP64 QR of tall panels (shifted Cholesky QR) and SVD of small square
// matrices (block one-sided Jacobi), batched over independent problems.
#pragma once

#include "common.hpp"
#include "gemm.hpp"

namespace ctm {

struct SmallLA {
  int kmax = 0, batch_max = 0;
  // flag: 256 ints; [0, 64) failure per problem (Cholesky breakdown, or a
  // Jacobi SVD that did not converge), [64, 128) Jacobi
  // convergence per problem, [128, 192) projector-weight failure per problem,
  // [192, 256) Jacobi sweeps run per problem
  DevBuf G, R, Rinv, Racc, Rtmp, J, flag, off, tmp, mask;
  PinnedBuf hflag;   // pinned staging of the convergence flags read by the host
  size_t tmp_elems = 0;
};

// True if order-k problems fit the workspaces and the LDS of the kernels below.
bool smallla_fits(const SmallLA& s, int k);

// Largest k (panel width / matrix order) the kernels below handle.
constexpr int kSmallLAMaxK = 320;
constexpr int kSvSmallMax = 128;   // largest matrix of singular_values_small

void smallla_alloc(SmallLA& s, int kmax, int batch_max, long nmax);

// Orthonormalise `batch` column-major n x k panels Y_b = Y + b * ystride in
// place by `passes` Cholesky QR passes, the first one with the shift of
// Fukaya et al. (2020) so that ill-conditioned panels stay positive
// definite.  If Racc != nullptr, Racc_b (k x k, col-major) receives the upper
// triangular factor with Y_in = Q R.  A pass whose Gram matrix has a
// non-finite pivot, or (from the third pass on) is far from the identity,
// sets flag[b] to 10 * pass + 1 or 10 * pass + 2 (device ints, one per
// problem; cleared by the caller).
void cholqr(hipStream_t st, SmallLA& s, double* Y, long ystride, int n, int k, int batch, int passes,
            double* Racc, const GemmWorkspace& ws);

// SVD of `batch` k x k column-major matrices A_b = X_b diag(S_b) Y_b^T by
// block one-sided Jacobi (A is overwritten).  S_b descending; X, Y k x k
// col-major, batch strides k*k; S_b = S + b * sstride (sstride >= k).
void jacobi_svd(hipStream_t st, SmallLA& s, double* A, int k, int batch, double* X, double* S, long sstride,
                double* Y);
// The same in two calls, so that other work can be enqueued between them:
// _start launches the sweeps that run before the first host read of the
// convergence flags; _finish reads them (synchronising st), runs the sweeps
// still needed and writes X, S, Y.
void jacobi_svd_start(hipStream_t st, SmallLA& s, double* A, int k, int batch);
void jacobi_svd_finish(hipStream_t st, SmallLA& s, double* A, int k, int batch, double* X, double* S, long sstride,
                       double* Y);

// Singular values (descending, m per problem at S + b * m) of `batch`
// column-major m x m matrices at A + b * m * m, m <= kSvSmallMax, by one-sided
// Jacobi in one workgroup per matrix (A is read, not changed).
void singular_values_small(hipStream_t st, const double* A, int m, int batch, double* S);
// The same for m x m matrices with m <= kSmallLAMaxK (batch <= 64), by the
// blocked one-sided Jacobi without rotation accumulation: A (column-major,
// b * m * m apart) is overwritten; S_b at S + b * sstride.  off, conv,
// nsweep: device workspaces of batch entries; hconv: pinned host ints.
void singular_values_batched(hipStream_t st, double* A, int m, int batch, double* S, long sstride, double* off,
                             int* conv, int* nsweep, int* hconv);

}  // namespace ctm
