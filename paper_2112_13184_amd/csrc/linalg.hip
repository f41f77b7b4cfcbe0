// FP64 factorisations on the GPU through rocSOLVER (Householder QR, SVD, symmetric eigenproblem).
#include "linalg.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "kernels.hpp"

namespace ctm {

struct Linalg {
  rocblas_handle h = nullptr;
  hipStream_t st = nullptr;
  DevBuf tau, info, E;
};

#define CTM_RB(call)                                                                          \
  do {                                                                                        \
    rocblas_status s_ = (call);                                                               \
    if (s_ != rocblas_status_success)                                                         \
      throw ::ctm::Error(-3, std::string(#call) + " failed: " + rocblas_status_to_string(s_)); \
  } while (0)

static constexpr int kMaxK = 4096;

Linalg* linalg_create(hipStream_t st) {
  Linalg* la = new Linalg();
  la->st = st;
  if (rocblas_create_handle(&la->h) != rocblas_status_success) {
    delete la;
    throw Error(-3, "rocblas_create_handle failed");
  }
  rocblas_set_stream(la->h, st);
  try {
    la->tau.alloc(kMaxK * sizeof(double));
    la->info.alloc(kMaxK * sizeof(rocblas_int));
    la->E.alloc((size_t)kMaxK * 64 * sizeof(double));
  } catch (...) {
    rocblas_destroy_handle(la->h);
    delete la;
    throw;
  }
  return la;
}

void linalg_destroy(Linalg* la) {
  if (!la) return;
  if (la->h) rocblas_destroy_handle(la->h);
  delete la;
}

void la_orth(Linalg* la, double* Y, int n, int k) {
  CTM_CHECK(n >= k && k <= kMaxK, -1, "la_orth: need n >= k and k <= 4096");
  CTM_RB(rocsolver_dgeqrf(la->h, n, k, Y, n, la->tau.as<double>()));
  CTM_RB(rocsolver_dorgqr(la->h, n, k, k, Y, n, la->tau.as<double>()));
}

void la_qr(Linalg* la, double* Z, int n, int k, double* R) {
  CTM_CHECK(n >= k && k <= kMaxK, -1, "la_qr: need n >= k and k <= 4096");
  CTM_RB(rocsolver_dgeqrf(la->h, n, k, Z, n, la->tau.as<double>()));
  extract_upper(la->st, Z, n, k, R);
  CTM_RB(rocsolver_dorgqr(la->h, n, k, k, Z, n, la->tau.as<double>()));
}

void la_svd(Linalg* la, double* A, int k, double* S, double* U, double* VT) {
  CTM_CHECK(k <= kMaxK, -1, "la_svd: k <= 4096");
  CTM_RB(rocsolver_dgesvd(la->h, rocblas_svect_singular, rocblas_svect_singular, k, k, A, k, S, U, k,
                          VT, k, la->E.as<double>(), rocblas_outofplace, la->info.as<rocblas_int>()));
}

void la_syev(Linalg* la, double* A, int n, double* W) {
  CTM_CHECK(n <= kMaxK, -1, "la_syev: n <= 4096");
  CTM_RB(rocsolver_dsyevd(la->h, rocblas_evect_original, rocblas_fill_lower, n, A, n, W, la->E.as<double>(),
                          la->info.as<rocblas_int>()));
}

void la_singular_values_batched(Linalg* la, double* A, int m, int batch, double* S) {
  CTM_CHECK(batch <= 64 && m <= kMaxK, -1, "la_singular_values_batched: batch <= 64");
  CTM_RB(rocsolver_dgesvd_strided_batched(
      la->h, rocblas_svect_none, rocblas_svect_none, m, m, A, m, (rocblas_stride)m * m, S,
      (rocblas_stride)m, nullptr, m, 0, nullptr, m, 0, la->E.as<double>(), (rocblas_stride)m,
      rocblas_outofplace, la->info.as<rocblas_int>(), batch));
}

}  // namespace ctm
