// Bandwidth-bound helper kernels of the CTMRG sweep.
#include "kernels.hpp"

#include <algorithm>
#include <cmath>

namespace ctm {
namespace {

constexpr int TPB = 256;

inline int grid_for(long n, int tpb = TPB, int cap = 8192) {
  long b = (n + tpb - 1) / tpb;
  return (int)std::max<long>(1, std::min<long>(b, cap));
}

__global__ void k_swap_last2(const double* in, double* out, long na, long nb, long nc) {
  long total = na * nb * nc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    // e indexes the output [a][c][b] so that writes are contiguous
    long b = e % nb;
    long t = e / nb;
    long c = t % nc;
    long a = t / nc;
    out[e] = in[(a * nb + b) * nc + c];
  }
}

struct PermArgs {
  int rank;
  long odims[12];    // output dims
  long istride[12];   // input stride of output axis k
};

__global__ void k_permute(const double* in, double* out, long total, PermArgs p) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long rem = e, src = 0;
    for (int k = p.rank - 1; k >= 0; --k) {
      long i = rem % p.odims[k];
      rem /= p.odims[k];
      src += i * p.istride[k];
    }
    out[e] = in[src];
  }
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = -1.0;
  if (threadIdx.x == 0) {
    r = sh[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
    sh[0] = r;
  }
  __syncthreads();
  r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    sh[0] = r;
  }
  __syncthreads();
  double r = sh[0];
  __syncthreads();
  return r;
}

// Partial max |x| per block; NaN recorded as +Inf so that it is caught.
__global__ void k_maxabs_partial(const double* x, long n, double* part) {
  __shared__ double sh[16];
  double m = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double v = fabs(x[i]);
    m = (v != v) ? INFINITY : fmax(m, v);
  }
  m = block_max(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void k_maxabs_final(double* part, int nparts, int* bad) {
  __shared__ double sh[16];
  double m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmax(m, part[i]);
  m = block_max(m, sh);
  if (threadIdx.x == 0) {
    part[1024] = m;
    if (!(m > 0.0) || !isfinite(m)) *bad = 1;
  }
}

__global__ void k_scale_by_inv(double* x, long n, const double* den) {
  double m = *den;
  if (!(m > 0.0) || !isfinite(m)) return;
  double inv = 1.0 / m;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] *= inv;
}

__global__ void k_identity_panel(double* P, int n, int chi, int nact) {
  long total = (long)n * chi;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int i = (int)(e / chi), k = (int)(e % chi);
    P[e] = (i == k && i < nact) ? 1.0 : 0.0;
  }
}

// Philox4x64-10 (Salmon et al., SC'11): two 64x64->128 multiplies per round,
// Weyl key schedule, ten rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__global__ void k_omega(double* Om, int n, int Db, int k, uint64_t seed, uint64_t sid) {
  // one thread per (row, group of 4 columns)
  int groups = (k + 3) / 4;
  long total = (long)n * groups;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int row = (int)(e % n);
    int g = (int)(e / n);
    uint64_t c[4] = {(uint64_t)(row / Db), (uint64_t)(row % Db), (uint64_t)g, sid};
    philox4x64_10(c, seed, 0ull);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      int j = 4 * g + w;
      if (j < k) Om[(long)j * n + row] = (double)(c[w] >> 11) * 0x1p-52 - 1.0;
    }
  }
}

// One block per projector column i < chi.
__global__ void k_projector_weights(const double* S, const double* U, int n, int kk, int chi, int kcap,
                                    double cutoff, double* w, int* bad) {
  __shared__ double shv[16];
  __shared__ int shi[16];
  int i = blockIdx.x;
  double s0 = S[0];
  if (i == 0 && threadIdx.x == 0 && (!(s0 > 0.0) || !isfinite(s0))) *bad = 1;
  bool keep = (i < kk) && (i < kcap) && (s0 > 0.0) && isfinite(s0) && (S[i] > cutoff * s0);
  if (!keep) {
    if (threadIdx.x == 0) w[i] = 0.0;
    return;
  }
  // argmax |U[:, i]|, first index on ties
  const double* u = U + (long)i * n;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double v = fabs(u[j]);
    if (v > best) { best = v; bi = j; }
  }
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    double ov = __shfl_xor(best, o);
    int oi = __shfl_xor(bi, o);
    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
  }
  if (lane == 0) { shv[wv] = best; shi[wv] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
      if (shv[q] > best || (shv[q] == best && shi[q] < bi)) { best = shv[q]; bi = shi[q]; }
    double sg = (u[bi] < 0.0) ? -1.0 : 1.0;
    w[i] = sg / sqrt(S[i]);
  }
}

__global__ void k_count_nonzero(const double* w, int chi, int* keff) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int c = 0;
    for (int i = 0; i < chi; ++i) c += (w[i] != 0.0);
    *keff = c;
  }
}

__global__ void k_scale_columns(double* X, int n, int m, const double* w) {
  long total = (long)n * m;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    X[e] *= w[e / n];
}

__global__ void k_extract_upper(const double* QR, int lda, int kk, double* R) {
  long total = (long)kk * kk;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int i = (int)(e % kk), j = (int)(e / kk);
    R[e] = (i <= j) ? QR[(long)j * lda + i] : 0.0;
  }
}

__global__ void k_transpose_square(const double* in, double* out, int kk) {
  long total = (long)kk * kk;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int i = (int)(e % kk), j = (int)(e / kk);
    out[(long)i * kk + j] = in[e];
  }
}

__global__ void k_spectra_delta(double* S, double* prev, int ncorner, int chi, double* delta) {
  __shared__ double sh[16];
  double dmax = 0.0;
  for (int c = 0; c < ncorner; ++c) {
    double* s = S + (long)c * chi;
    double part = 0.0;
    for (int i = threadIdx.x; i < chi; i += blockDim.x) part += s[i];
    double tot = block_sum(part, sh);
    double inv = (tot > 0.0) ? 1.0 / tot : 0.0;
    double dl = 0.0;
    for (int i = threadIdx.x; i < chi; i += blockDim.x) {
      double v = s[i] * inv;
      dl += fabs(v - prev[(long)c * chi + i]);
      s[i] = v;
      prev[(long)c * chi + i] = v;
    }
    double d = block_sum(dl, sh);
    dmax = fmax(dmax, d);
  }
  if (threadIdx.x == 0) *delta = dmax;
}

__global__ void k_scale(double* x, long n, double a) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] *= a;
}

// ---- batched forms: problem b = blockIdx.y, its own pointers ---------------

constexpr int kMaxBatchArgs = 64;   // per-problem scalars passed by value

__global__ void k_swap_last2_b(const double* const* in, double* const* out, long na, long nb, long nc) {
  const double* src = in[blockIdx.y];
  double* dst = out[blockIdx.y];
  long total = na * nb * nc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long b = e % nb;
    long t = e / nb;
    long c = t % nc;
    long a = t / nc;
    dst[e] = src[(a * nb + b) * nc + c];
  }
}

// part: kNormSlots doubles per problem (block maxima, then the maximum at 1024)
constexpr int kNormSlots = 1025;

__global__ void k_maxabs_partial_b(double* const* x, long n, double* part) {
  __shared__ double sh[16];
  const double* xb = x[blockIdx.y];
  double m = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double v = fabs(xb[i]);
    m = (v != v) ? INFINITY : fmax(m, v);
  }
  m = block_max(m, sh);
  if (threadIdx.x == 0) part[(long)blockIdx.y * kNormSlots + blockIdx.x] = m;
}

__global__ void k_maxabs_final_b(double* part, int nparts, int* bad, const long* flag_index) {
  __shared__ double sh[16];
  double* pb = part + (long)blockIdx.x * kNormSlots;
  double m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmax(m, pb[i]);
  m = block_max(m, sh);
  if (threadIdx.x == 0) {
    pb[1024] = m;
    if (!(m > 0.0) || !isfinite(m)) bad[flag_index ? flag_index[blockIdx.x] : 0] = 1;
  }
}

__global__ void k_scale_by_inv_b(double* const* x, long n, const double* part) {
  double m = part[(long)blockIdx.y * kNormSlots + 1024];
  if (!(m > 0.0) || !isfinite(m)) return;
  double inv = 1.0 / m;
  double* xb = x[blockIdx.y];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) xb[i] *= inv;
}

struct OmegaKeys {
  uint64_t seed[kMaxBatchArgs], sid[kMaxBatchArgs];
};

__global__ void k_omega_b(double* Om, long ostride, int n, int Db, int k, OmegaKeys keys) {
  const int b = blockIdx.y;
  double* O = Om + (long)b * ostride;
  const uint64_t sd = keys.seed[b], si = keys.sid[b];
  int groups = (k + 3) / 4;
  long total = (long)n * groups;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int row = (int)(e % n);
    int g = (int)(e / n);
    uint64_t c[4] = {(uint64_t)(row / Db), (uint64_t)(row % Db), (uint64_t)g, si};
    philox4x64_10(c, sd, 0ull);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      int j = 4 * g + w;
      if (j < k) O[(long)j * n + row] = (double)(c[w] >> 11) * 0x1p-52 - 1.0;
    }
  }
}

struct Caps {
  int v[kMaxBatchArgs];
};

__global__ void k_projector_weights_b(const double* S, long sstride, const double* U, long ustride, int n, int kk,
                                      int chi, Caps kcap, double cutoff, double* w, int* bad) {
  // one block per (column i, problem b): the single form on problem b's data
  __shared__ double shv[16];
  __shared__ int shi[16];
  const int b = blockIdx.y, i = blockIdx.x;
  const double* Sb = S + (long)b * sstride;
  double* wb = w + (long)b * chi;
  double s0 = Sb[0];
  if (i == 0 && threadIdx.x == 0 && (!(s0 > 0.0) || !isfinite(s0))) bad[b] = 1;
  bool keep = (i < kk) && (i < kcap.v[b]) && (s0 > 0.0) && isfinite(s0) && (Sb[i] > cutoff * s0);
  if (!keep) {
    if (threadIdx.x == 0) wb[i] = 0.0;
    return;
  }
  const double* u = U + (long)b * ustride + (long)i * n;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double v = fabs(u[j]);
    if (v > best) { best = v; bi = j; }
  }
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    double ov = __shfl_xor(best, o);
    int oi = __shfl_xor(bi, o);
    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
  }
  if (lane == 0) { shv[wv] = best; shi[wv] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
      if (shv[q] > best || (shv[q] == best && shi[q] < bi)) { best = shv[q]; bi = shi[q]; }
    double sg = (u[bi] < 0.0) ? -1.0 : 1.0;
    wb[i] = sg / sqrt(Sb[i]);
  }
}

__global__ void k_count_nonzero_b(const double* w, int chi, int* keff, int batch) {
  const int b = threadIdx.x;
  if (b < batch) {
    int c = 0;
    for (int i = 0; i < chi; ++i) c += (w[(long)b * chi + i] != 0.0);
    keff[b] = c;
  }
}

__global__ void k_scale_columns_b(double* X, long xstride, int n, int m, const double* w, long wstride) {
  double* Xb = X + (long)blockIdx.y * xstride;
  const double* wb = w + (long)blockIdx.y * wstride;
  long total = (long)n * m;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    Xb[e] *= wb[e / n];
}

__global__ void k_transpose_square_b(const double* in, double* out, int kk) {
  const long off = (long)blockIdx.y * kk * kk;
  long total = (long)kk * kk;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int i = (int)(e % kk), j = (int)(e / kk);
    out[off + (long)i * kk + j] = in[off + e];
  }
}

}  // namespace

void swap_last2(hipStream_t st, const double* in, double* out, long na, long nb, long nc) {
  long total = na * nb * nc;
  hipLaunchKernelGGL(k_swap_last2, dim3(grid_for(total)), dim3(TPB), 0, st, in, out, na, nb, nc);
  CTM_HIP(hipGetLastError());
}

void permute(hipStream_t st, const double* in, double* out, int rank, const long* dims, const int* perm) {
  CTM_CHECK(rank >= 1 && rank <= 12, -1, "permute: rank must be 1..12");
  long istr[12];
  long s = 1;
  for (int k = rank - 1; k >= 0; --k) { istr[k] = s; s *= dims[k]; }
  PermArgs p{};
  p.rank = rank;
  long total = 1;
  for (int k = 0; k < rank; ++k) {
    p.odims[k] = dims[perm[k]];
    p.istride[k] = istr[perm[k]];
    total *= p.odims[k];
  }
  hipLaunchKernelGGL(k_permute, dim3(grid_for(total)), dim3(TPB), 0, st, in, out, total, p);
  CTM_HIP(hipGetLastError());
}

void normalize_maxabs(hipStream_t st, double* x, long n, double* scratch, int* bad_flag) {
  int nb = std::min(1024, grid_for(n));
  hipLaunchKernelGGL(k_maxabs_partial, dim3(nb), dim3(TPB), 0, st, x, n, scratch);
  hipLaunchKernelGGL(k_maxabs_final, dim3(1), dim3(TPB), 0, st, scratch, nb, bad_flag);
  hipLaunchKernelGGL(k_scale_by_inv, dim3(grid_for(n)), dim3(TPB), 0, st, x, n, scratch + 1024);
  CTM_HIP(hipGetLastError());
}

void identity_panel(hipStream_t st, double* P, int n, int chi, int nact) {
  hipLaunchKernelGGL(k_identity_panel, dim3(grid_for((long)n * chi)), dim3(TPB), 0, st, P, n, chi, nact);
  CTM_HIP(hipGetLastError());
}

void omega_fill(hipStream_t st, double* Om, int n, int Db, int k, uint64_t seed, uint64_t sid) {
  long total = (long)n * ((k + 3) / 4);
  hipLaunchKernelGGL(k_omega, dim3(grid_for(total)), dim3(TPB), 0, st, Om, n, Db, k, seed, sid);
  CTM_HIP(hipGetLastError());
}

void projector_weights(hipStream_t st, const double* S, const double* U, int n, int kk, int chi,
                       int kcap, double cutoff, double* w, int* keff, int* bad_flag) {
  hipLaunchKernelGGL(k_projector_weights, dim3(chi), dim3(TPB), 0, st, S, U, n, kk, chi, kcap, cutoff, w, bad_flag);
  hipLaunchKernelGGL(k_count_nonzero, dim3(1), dim3(64), 0, st, w, chi, keff);
  CTM_HIP(hipGetLastError());
}

void scale_columns(hipStream_t st, double* X, int n, int m, const double* w) {
  hipLaunchKernelGGL(k_scale_columns, dim3(grid_for((long)n * m)), dim3(TPB), 0, st, X, n, m, w);
  CTM_HIP(hipGetLastError());
}

void extract_upper(hipStream_t st, const double* QR, int lda, int kk, double* R) {
  hipLaunchKernelGGL(k_extract_upper, dim3(grid_for((long)kk * kk)), dim3(TPB), 0, st, QR, lda, kk, R);
  CTM_HIP(hipGetLastError());
}

void transpose_square(hipStream_t st, const double* in, double* out, int kk) {
  hipLaunchKernelGGL(k_transpose_square, dim3(grid_for((long)kk * kk)), dim3(TPB), 0, st, in, out, kk);
  CTM_HIP(hipGetLastError());
}

void spectra_delta(hipStream_t st, double* S, double* prev, int ncorner, int chi, double* delta_out) {
  hipLaunchKernelGGL(k_spectra_delta, dim3(1), dim3(TPB), 0, st, S, prev, ncorner, chi, delta_out);
  CTM_HIP(hipGetLastError());
}

void scale_by_inv(hipStream_t st, double* x, long n, const double* den) {
  hipLaunchKernelGGL(k_scale_by_inv, dim3(grid_for(n)), dim3(TPB), 0, st, x, n, den);
  CTM_HIP(hipGetLastError());
}

void scale(hipStream_t st, double* x, long n, double a) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(TPB), 0, st, x, n, a);
  CTM_HIP(hipGetLastError());
}


void swap_last2_batched(hipStream_t st, const double* const* in, double* const* out, int batch, long na, long nb,
                        long nc) {
  if (batch <= 0) return;
  long total = na * nb * nc;
  hipLaunchKernelGGL(k_swap_last2_b, dim3(std::max(1, grid_for(total) / batch), batch), dim3(TPB), 0, st, in, out, na,
                     nb, nc);
  CTM_HIP(hipGetLastError());
}

void normalize_maxabs_batched(hipStream_t st, double* const* x, int batch, long n, double* scratch, int* bad_flag,
                              const long* flag_index) {
  if (batch <= 0) return;
  int nb = std::min(1024, grid_for(n));
  hipLaunchKernelGGL(k_maxabs_partial_b, dim3(nb, batch), dim3(TPB), 0, st, x, n, scratch);
  hipLaunchKernelGGL(k_maxabs_final_b, dim3(batch), dim3(TPB), 0, st, scratch, nb, bad_flag, flag_index);
  hipLaunchKernelGGL(k_scale_by_inv_b, dim3(grid_for(n), batch), dim3(TPB), 0, st, x, n, scratch);
  CTM_HIP(hipGetLastError());
}

void omega_fill_batched(hipStream_t st, double* Om, long ostride, int batch, int n, int Db, int k, const uint64_t* seed,
                        const uint64_t* sid) {
  if (batch <= 0) return;
  CTM_CHECK(batch <= kMaxBatchArgs, -1, "omega_fill_batched: at most 64 problems");
  OmegaKeys keys{};
  for (int b = 0; b < batch; ++b) {
    keys.seed[b] = seed[b];
    keys.sid[b] = sid[b];
  }
  long total = (long)n * ((k + 3) / 4);
  hipLaunchKernelGGL(k_omega_b, dim3(grid_for(total), batch), dim3(TPB), 0, st, Om, ostride, n, Db, k, keys);
  CTM_HIP(hipGetLastError());
}

void scale_columns_batched(hipStream_t st, double* X, long xstride, int batch, int n, int m, const double* w,
                           long wstride) {
  if (batch <= 0) return;
  hipLaunchKernelGGL(k_scale_columns_b, dim3(grid_for((long)n * m), batch), dim3(TPB), 0, st, X, xstride, n, m, w,
                     wstride);
  CTM_HIP(hipGetLastError());
}

void transpose_square_batched(hipStream_t st, const double* in, double* out, int kk, int batch) {
  if (batch <= 0) return;
  hipLaunchKernelGGL(k_transpose_square_b, dim3(grid_for((long)kk * kk), batch), dim3(TPB), 0, st, in, out, kk);
  CTM_HIP(hipGetLastError());
}


void projector_weights_batched(hipStream_t st, const double* S, long sstride, const double* U, long ustride, int n,
                               int kk, int chi, const int* kcap, double cutoff, double* w, int* keff, int* bad_flag,
                               int batch) {
  if (batch <= 0) return;
  CTM_CHECK(batch <= kMaxBatchArgs, -1, "projector_weights_batched: at most 64 problems");
  Caps caps{};
  for (int b = 0; b < batch; ++b) caps.v[b] = kcap[b];
  hipLaunchKernelGGL(k_projector_weights_b, dim3(chi, batch), dim3(TPB), 0, st, S, sstride, U, ustride, n, kk, chi,
                     caps, cutoff, w, bad_flag);
  hipLaunchKernelGGL(k_count_nonzero_b, dim3(1), dim3(1024), 0, st, w, chi, keff, batch);
  CTM_HIP(hipGetLastError());
}

}  // namespace ctm
