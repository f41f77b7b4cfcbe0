// Small device kernels of the CTMRG sweep (bandwidth-bound helpers).
#pragma once

#include "common.hpp"

namespace ctm {

// out[a][c][b] = in[a][b][c] for dims (na, nb, nc).
void swap_last2(hipStream_t st, const double* in, double* out, long na, long nb, long nc);

// General permutation of an up-to-12-dimensional row-major tensor:
// out[i_perm[0]]...[i_perm[r-1]] = in[i_0]...[i_{r-1}], i.e. out axis k is in axis perm[k].
void permute(hipStream_t st, const double* in, double* out, int rank, const long* dims, const int* perm);

// x /= max|x| over n entries (FP64).  scratch: >= 1024 doubles.  Also sets
// *bad_flag (device int) to 1 if the maximum is 0, NaN or Inf.
void normalize_maxabs(hipStream_t st, double* x, long n, double* scratch, int* bad_flag);

// Panel P (n x chi, row-major) = identity on the first nact rows / columns.
void identity_panel(hipStream_t st, double* P, int n, int chi, int nact);

// Sketch matrix (column-major, ld = n) of Philox4x64-10 uniforms on [-1, 1):
// entry (row = c*Db + b, col j) from counter (c, b, j/4, sid), key (seed, 0).
void omega_fill(hipStream_t st, double* Om, int n, int Db, int k, uint64_t seed, uint64_t sid);

// Projector scaling after the small SVD.  Given S (kk values, descending),
// U (n x kk, col-major, the left singular vectors whose largest-|.| entry
// fixes the sign) computes w[i] = sign_i / sqrt(S_i) for i < min(chi, kk, kcap)
// with S_i > cutoff * S_0, else 0, for i < chi; writes k_eff to *keff.
// kcap is the structural rank bound of the cut (smallest bond of the product).
void projector_weights(hipStream_t st, const double* S, const double* U, int n, int kk, int chi,
                       int kcap, double cutoff, double* w, int* keff, int* bad_flag);

// X[:, j] *= w[j] for a column-major n x m panel (ld = n), columns j < m.
void scale_columns(hipStream_t st, double* X, int n, int m, const double* w);

// Copy the upper triangle of a column-major kk x kk block (ld = lda) into R
// (col-major, ld = kk), zeros below the diagonal.
void extract_upper(hipStream_t st, const double* QR, int lda, int kk, double* R);

// Column-major kk x kk: out = in^T.
void transpose_square(hipStream_t st, const double* in, double* out, int kk);

// Corner spectra: S (ncorner x chi) -> normalised to sum 1; delta = max over
// corners of sum |s - prev|; prev <- s.  delta_out: one device double.
void spectra_delta(hipStream_t st, double* S, double* prev, int ncorner, int chi, double* delta_out);

// y[i] = a * x[i]
void scale(hipStream_t st, double* x, long n, double a);

// x /= *den (a device scalar, e.g. the maximum normalize_maxabs leaves in
// scratch[1024]); no change if *den is 0 or not finite.
void scale_by_inv(hipStream_t st, double* x, long n, const double* den);


// Batched forms for problems of one shape in one launch (problem b on
// blockIdx.y).  Pointer arguments of type `T* const*` are device arrays of one
// device pointer per problem; strides are in elements.  Each problem gets
// exactly the arithmetic of the single form.
void swap_last2_batched(hipStream_t st, const double* const* in, double* const* out, int batch, long na, long nb,
                        long nc);
// scratch: 1025 doubles per problem.  A problem whose maximum is 0, NaN or
// Inf sets bad_flag[flag_index[b]] (device array; bad_flag[0] when
// flag_index is null).
void normalize_maxabs_batched(hipStream_t st, double* const* x, int batch, long n, double* scratch, int* bad_flag,
                              const long* flag_index = nullptr);
// Problem b: Om + b * ostride, key seed[b], stream id sid[b] (host arrays,
// batch <= 64).
void omega_fill_batched(hipStream_t st, double* Om, long ostride, int batch, int n, int Db, int k, const uint64_t* seed,
                        const uint64_t* sid);
void scale_columns_batched(hipStream_t st, double* X, long xstride, int batch, int n, int m, const double* w,
                           long wstride);
// Problem b: in / out + b * kk * kk.
void transpose_square_batched(hipStream_t st, const double* in, double* out, int kk, int batch);

// Problem b: S + b * sstride, U + b * ustride, cap kcap[b] (host array,
// batch <= 64), weights w + b * chi, keff[b], bad_flag[b].
void projector_weights_batched(hipStream_t st, const double* S, long sstride, const double* U, long ustride, int n,
                               int kk, int chi, const int* kcap, double cutoff, double* w, int* keff, int* bad_flag,
                               int batch);

}  // namespace ctm
