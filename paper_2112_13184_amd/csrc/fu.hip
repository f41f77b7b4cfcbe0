// Full-update imaginary-time evolution (Sec. 2.3, Eq. (4) with the CTMRG
// environment; Jordan et al. 2008 in the reduced-tensor form of Phien et al.
// 2015).  One bond update (i, j) of the site tensors held by a CTMRG context,
// with that context's current environment:
//   1. A_i as [(three other legs), (bond k, p)] = X_i a_i (Householder QR),
//      likewise j;
//   2. the bond environment N[(rho_i rho_j)][(rho_i' rho_j')]: the bond
//      density-matrix patch with X_i, X_j in place of the sites (their bond
//      leg pinned to one index, so the bond is cut) and the reduced legs open,
//      trace 1 (observe.hip, bond_environment);
//   3. N <- the positive part of (N + N^T) / 2 (eigendecomposition);
//   4. Theta'[(rho_i P)][(rho_j Q)] = sum_{pq} g[(P Q)][(p q)] sum_k a_i[rho_i][(k p)] a_j[rho_j][(k q)];
//   5. start from the truncated SVD of Theta' (sqrt of the singular values
//      on both factors);
//   6. alternating least squares: each factor solves its quadratic
//      subproblem R x = S through the pseudo-inverse of R (eigenvalues
//      <= 1e-12 of the largest dropped);
//   7. A_i' = X_i b_i, A_j' = X_j b_j back in [l][u][r][d][p]; the sign of
//      each bond index makes the first entry of A_i'[.., k, ..] within 1e-8
//      of its largest modulus positive (A_j' flipped with it); each tensor is
//      divided by its largest |entry|; all four rotations are rewritten;
//   8. env_sweeps CTMRG sweeps from the current environment.
// Every step runs on the context's stream.  The QRs (up to 8192 entries) and
// the symmetric eigenproblems (up to order 64) are one-workgroup kernels
// here, larger ones and the SVD of step 5 go through rocSOLVER; the
// contractions through the FP64 MFMA GEMM.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "context.hpp"
#include "gemm.hpp"
#include "linalg.hpp"
#include "wave.hpp"

namespace ctm {
namespace {

constexpr double kFuPinvCut = 1e-12;
constexpr double kFuSignTol = 1e-8;

__device__ inline int fu_other_leg(int leg, int t) {
  return t == 0 ? (leg == 0 ? 1 : 0) : t == 1 ? (leg <= 1 ? 2 : 1) : (leg <= 2 ? 3 : 2);
}

// out[l][u][r][d][rho] = Q(alpha, rho) where leg `leg` is 0 (alpha: the other
// three legs in order), else 0; Q column-major R3 x r.
__global__ void k_fu_embed(const double* Q, double* out, int D, int r, int leg) {
  const long R3 = (long)D * D * D, total = R3 * D * r;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int rho = (int)(e % r);
    const long t = e / r;
    const int l3 = (int)(t % D), l2 = (int)((t / D) % D), l1 = (int)((t / ((long)D * D)) % D),
              l0 = (int)(t / ((long)D * D * D));
    const int pinned = leg == 0 ? l0 : leg == 1 ? l1 : leg == 2 ? l2 : l3;
    double v = 0.0;
    if (pinned == 0) {
      const int o0 = leg == 0 ? l1 : l0;
      const int o1 = leg <= 1 ? l2 : l1;
      const int o2 = leg <= 2 ? l3 : l2;
      v = Q[((long)o0 * D + o1) * D + o2 + (long)rho * R3];
    }
    out[e] = v;
  }
}

// B = (A + A^T) / 2, n x n
__global__ void k_fu_sym(const double* A, double* B, int n) {
  const long total = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    B[e] = 0.5 * (A[(long)i * n + j] + A[(long)j * n + i]);
  }
}

// Vs = V diag(max(w, 0)) (V column-major n x n)
__global__ void k_fu_pos_cols(const double* V, const double* w, double* Vs, int n) {
  const long total = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int col = (int)(e / n);
    Vs[e] = V[e] * fmax(w[col], 0.0);
  }
}

// Y[i][:] *= 1 / w_i where w_i > cut * max(w_max, 0), else 0 (w in any order)
__global__ void k_fu_pinv_rows(double* Y, const double* w, int n, int m) {
  double wmax = 0.0;                               // the largest eigenvalue (any order)
  for (int i = 0; i < n; ++i) wmax = fmax(wmax, w[i]);
  const long total = (long)n * m;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / m);
    const double wi = w[i];
    Y[e] = wi > kFuPinvCut * wmax ? Y[e] / wi : 0.0;
  }
}

// Eigen-decomposition of one symmetric n x n matrix (n <= kFuEigMax) in one
// workgroup by the cyclic two-sided Jacobi method: each round applies the
// n / 2 rotations of a round-robin tournament of disjoint index pairs
// (p, q) together, A <- J^T A J with J the rotation that zeroes a_pq of the
// pair's 2 x 2 block (t = sgn(z) / (|z| + sqrt(z^2 + 1)), z = (a_qq - a_pp) /
// (2 a_pq), c = 1 / sqrt(t^2 + 1), s = t c), rows first, then columns and
// the accumulated V <- V J.  An entry is rotated away while |a_pq| exceeds
// 1e-16 ||A||_F; the iteration ends after a sweep with no rotation (or
// after kFuEigMaxSweeps).  A (column-major, symmetric) is read; W receives
// the eigenvalues (unsorted) and V the eigenvectors (column j for W[j],
// column-major n x n).  *unconverged is set when the sweep cap is reached.
constexpr int kFuEigMax = 64;
constexpr int kFuEigLd = kFuEigMax + 1;
constexpr int kFuEigMaxSweeps = 30;

__device__ __forceinline__ int eig_circle(int pos, int round, int m) {
  if (pos == 0) return 0;
  int t = pos - 1 + round;
  if (t >= m - 1) t -= m - 1;
  return t + 1;
}

__global__ __launch_bounds__(1024) void k_sym_eig(const double* A, int n, double* W, double* V, int* unconverged) {
  __shared__ double a[kFuEigMax * kFuEigLd];
  __shared__ double v[kFuEigMax * kFuEigLd];
  __shared__ double cs[kFuEigMax / 2], sn[kFuEigMax / 2];
  __shared__ int pp[kFuEigMax / 2], qq[kFuEigMax / 2];
  __shared__ double red[16];
  __shared__ int rotated;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  const int m = n + (n & 1), half = m / 2;
  // a[i + kFuEigLd j] = A(i, j), zero in the padding row and column; v = I
  double f2 = 0.0;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    const double x = (i < n && j < n) ? A[i + (long)j * n] : 0.0;
    a[i + kFuEigLd * j] = x;
    v[i + kFuEigLd * j] = (i == j) ? 1.0 : 0.0;
    f2 += x * x;
  }
  f2 = wave_sum(f2);
  if (lane == 0) red[w] = f2;
  __syncthreads();
  double fro2 = 0.0;
  for (int i = 0; i < nw; ++i) fro2 += red[i];
  const double thr = 1e-16 * sqrt(fro2);
  int sw = 0;
  for (; sw < kFuEigMaxSweeps; ++sw) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      if (tid < half) {
        int p = eig_circle(tid, round, m), q = eig_circle(m - 1 - tid, round, m);
        if (p > q) { const int t = p; p = q; q = t; }
        const double apq = a[p + kFuEigLd * q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > thr) {
          const double z = (a[q + kFuEigLd * q] - a[p + kFuEigLd * p]) / (2.0 * apq);
          const double t = fabs(z) > 1e150 ? 0.5 / z : (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(z * z + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          rotated = 1;
        }
        pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
      }
      __syncthreads();
      // rows p, q of A
      for (int e = tid; e < half * m; e += blockDim.x) {
        const int k = e / m, j = e % m;
        const double c = cs[k], s = sn[k];
        if (s != 0.0) {
          const int p = pp[k], q = qq[k];
          const double x = a[p + kFuEigLd * j], y = a[q + kFuEigLd * j];
          a[p + kFuEigLd * j] = c * x - s * y;
          a[q + kFuEigLd * j] = s * x + c * y;
        }
      }
      __syncthreads();
      // columns p, q of A and of V
      for (int e = tid; e < half * m; e += blockDim.x) {
        const int k = e / m, i = e % m;
        const double c = cs[k], s = sn[k];
        if (s != 0.0) {
          const int p = pp[k], q = qq[k];
          const double x = a[i + kFuEigLd * p], y = a[i + kFuEigLd * q];
          a[i + kFuEigLd * p] = c * x - s * y;
          a[i + kFuEigLd * q] = s * x + c * y;
          const double u = v[i + kFuEigLd * p], z = v[i + kFuEigLd * q];
          v[i + kFuEigLd * p] = c * u - s * z;
          v[i + kFuEigLd * q] = s * u + c * z;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;
    V[e] = v[i + kFuEigLd * j];
  }
  for (int j = tid; j < n; j += blockDim.x) W[j] = a[j + kFuEigLd * j];
  if (tid == 0 && unconverged) *unconverged = sw == kFuEigMaxSweeps ? 1 : 0;
}

// Householder QR of one tall n x k matrix (column-major, n >= k, n k <=
// kQrMaxElems) in one workgroup, as LAPACK's geqr2 and org2r: reflector j
// has v = (1, x / (alpha - beta)), beta = -sgn(alpha) sqrt(alpha^2 + |x|^2),
// tau = (beta - alpha) / beta (tau = 0 when x = 0), applied to the columns
// right of j (one wave per column); then Q is formed in place from the
// reflectors in reverse order.  Z receives Q (n x k), R the k x k upper
// triangle (column-major).
constexpr int kQrMaxElems = 8192;
constexpr int kQrMaxK = 64;

__device__ double qr_block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += red[i];
  return r;
}

// H = I - tau v v^T (v_j = 1, v_i = a[i + n j] below j) on columns j+1..k-1
__device__ void qr_apply_right_of(double* a, int n, int k, int j, double tau) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (tau == 0.0) return;
  for (int c = j + 1 + w; c < k; c += nw) {
    double dot = 0.0;
    for (int i = j + 1 + lane; i < n; i += 64) dot += a[i + n * j] * a[i + n * c];
    dot = wave_sum(dot) + a[j + n * c];
    const double f = tau * dot;
    if (lane == 0) a[j + n * c] -= f;
    for (int i = j + 1 + lane; i < n; i += 64) a[i + n * c] -= f * a[i + n * j];
  }
}

__global__ __launch_bounds__(256) void k_small_qr(double* Z, int n, int k, double* R) {
  __shared__ double a[kQrMaxElems];
  __shared__ double tau[kQrMaxK];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  for (int e = tid; e < n * k; e += blockDim.x) a[e] = Z[e];
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    double x2 = 0.0;
    for (int i = j + 1 + tid; i < n; i += blockDim.x) x2 += a[i + n * j] * a[i + n * j];
    x2 = qr_block_sum(x2, red);
    const double alpha = a[j + n * j];
    double t = 0.0;
    if (x2 > 0.0) {
      const double beta = -copysign(sqrt(alpha * alpha + x2), alpha);
      t = (beta - alpha) / beta;
      const double sc = 1.0 / (alpha - beta);
      for (int i = j + 1 + tid; i < n; i += blockDim.x) a[i + n * j] *= sc;
      __syncthreads();
      if (tid == 0) a[j + n * j] = beta;
    }
    if (tid == 0) tau[j] = t;
    __syncthreads();
    qr_apply_right_of(a, n, k, j, t);
    __syncthreads();
  }
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int r = e % k, c = e / k;
    R[e] = r <= c ? a[r + n * c] : 0.0;
  }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double t = tau[j];
    if (j < k - 1) qr_apply_right_of(a, n, k, j, t);
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      if (i > j) a[i + n * j] *= -t;
      else if (i == j) a[i + n * j] = 1.0 - t;
      else a[i + n * j] = 0.0;
    }
    __syncthreads();
  }
  for (int e = tid; e < n * k; e += blockDim.x) Z[e] = a[e];
}

// Theta'[(x P)][(y Q)], a_i(x, c) = Ri[x + c C] (column-major C x C), likewise a_j
__global__ void k_fu_core(const double* Ri, const double* Rj, const double* g, double* Th, int D, int d, int C) {
  const int n = C * d;
  const long total = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int row = (int)(e / n), col = (int)(e % n);
    const int x = row / d, P = row % d, y = col / d, Q = col % d;
    double v = 0.0;
    for (int p = 0; p < d; ++p)
      for (int q = 0; q < d; ++q) {
        const double gv = g[(P * d + Q) * d * d + p * d + q];
        double t = 0.0;
        for (int k = 0; k < D; ++k) t += Ri[x + (long)(k * d + p) * C] * Rj[y + (long)(k * d + q) * C];
        v += gv * t;
      }
    Th[e] = v;
  }
}

// b_i[(x P)][k] = U_Th(row, k) sqrt(S_k), b_j[(y Q)][k] = V_Th(row, k) sqrt(S_k);
// the SVD was taken of Th^T (column-major view of the row-major Th), so U_Th
// is its VT and V_Th its U.
__global__ void k_fu_start(const double* Ucm, const double* VTcm, const double* S, double* bi, double* bj, int n,
                           int D) {
  const long total = (long)n * D;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int row = (int)(e / D), k = (int)(e % D);
    const double sq = sqrt(S[k]);
    bi[e] = VTcm[k + (long)row * n] * sq;
    bj[e] = Ucm[row + (long)k * n] * sq;
  }
}

// Sign rule and normalisation of the updated pair (one workgroup).
__global__ __launch_bounds__(256) void k_fu_sign_normalize(double* Ai, double* Aj, int D, int d, int li, int lj) {
  __shared__ double red[256];
  __shared__ int ired[256];
  __shared__ double flip[8];
  const int tid = threadIdx.x;
  const long per = (long)D * D * D * d, total = per * D;
  auto stride = [&](int leg) -> long {
    return leg == 0 ? (long)D * D * D * d : leg == 1 ? (long)D * D * d : leg == 2 ? (long)D * d : (long)d;
  };
  // element f (C order over the other three legs and p) of bond index k of A_i
  auto idx_i = [&](long f, int k) -> long {
    const int p = (int)(f % d);
    const long t = f / d;
    const int a3 = (int)(t % D), a2 = (int)((t / D) % D), a1 = (int)(t / ((long)D * D));
    return a1 * stride(fu_other_leg(li, 0)) + a2 * stride(fu_other_leg(li, 1)) + a3 * stride(fu_other_leg(li, 2)) +
           k * stride(li) + p;
  };
  for (int k = 0; k < D; ++k) {
    double m = 0.0;
    for (long f = tid; f < per; f += 256) m = fmax(m, fabs(Ai[idx_i(f, k)]));
    red[tid] = m;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
      __syncthreads();
    }
    const double thr = (1.0 - kFuSignTol) * red[0];
    int best = 1 << 30;
    for (long f = tid; f < per; f += 256)
      if (fabs(Ai[idx_i(f, k)]) >= thr) { best = (int)f; break; }
    __syncthreads();
    ired[tid] = best;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (tid < h) ired[tid] = min(ired[tid], ired[tid + h]);
      __syncthreads();
    }
    if (tid == 0) flip[k] = (red[0] > 0.0 && ired[0] < (1 << 30) && Ai[idx_i(ired[0], k)] < 0.0) ? -1.0 : 1.0;
    __syncthreads();
  }
  double mi = 0.0, mj = 0.0;
  for (long e = tid; e < total; e += 256) {
    const int ki = (int)((e / stride(li)) % D), kj = (int)((e / stride(lj)) % D);
    Ai[e] *= flip[ki];
    Aj[e] *= flip[kj];
    mi = fmax(mi, fabs(Ai[e]));
    mj = fmax(mj, fabs(Aj[e]));
  }
  red[tid] = mi;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const double si = red[0];
  __syncthreads();
  red[tid] = mj;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const double sj = red[0];
  for (long e = tid; e < total; e += 256) {
    if (si > 0.0) Ai[e] /= si;
    if (sj > 0.0) Aj[e] /= sj;
  }
}

int blocks_for(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 2048)); }

DT dt(double* p, std::vector<long> dims) {
  DT t;
  t.p = p;
  t.dims = std::move(dims);
  return t;
}

int other_leg_h(int leg, int t) { return t == 0 ? (leg == 0 ? 1 : 0) : t == 1 ? (leg <= 1 ? 2 : 1) : (leg <= 2 ? 3 : 2); }

// X = pinv(sym(Rm)) Sm, Rm n x n, Sm n x m (row-major, arena)
// Eigenvalues W and eigenvectors (columns of V, in place) of the symmetric
// n x n matrix V: one-workgroup Jacobi up to kFuEigMax, else rocSOLVER.
void sym_eig(Context& c, double* V, int n, double* W) {
  if (n <= kFuEigMax) {
    hipLaunchKernelGGL(k_sym_eig, dim3(1), dim3(1024), 0, c.st, V, n, W, V, nullptr);
    CTM_HIP(hipGetLastError());
  } else {
    la_syev(c.la, V, n, W);
  }
}

// Z (n x k) <- Q, R <- the k x k factor: one workgroup up to n k = kQrMaxElems,
// else rocSOLVER.
void small_qr(Context& c, double* Z, int n, int k, double* R) {
  if ((long)n * k <= kQrMaxElems && k <= kQrMaxK && n >= k) {
    hipLaunchKernelGGL(k_small_qr, dim3(1), dim3(256), 0, c.st, Z, n, k, R);
    CTM_HIP(hipGetLastError());
  } else {
    la_qr(c.la, Z, n, k, R);
  }
}

double* pinv_solve(Context& c, const double* Rm, const double* Sm, int n, int m) {
  double* V = c.arena.alloc((size_t)n * n);
  double* W = c.arena.alloc(n);
  double* Y = c.arena.alloc((size_t)n * m);
  double* X = c.arena.alloc((size_t)n * m);
  hipLaunchKernelGGL(k_fu_sym, dim3(blocks_for((long)n * n)), dim3(256), 0, c.st, Rm, V, n);
  CTM_HIP(hipGetLastError());
  sym_eig(c, V, n, W);                                           // V <- eigenvectors (columns)
  gemm(c.st, GemmType::F64, n, m, n, 1.0, rowmajor(V, n), rowmajor(Sm, m), 0.0, out_rowmajor(Y, m), 1, c.ws());
  hipLaunchKernelGGL(k_fu_pinv_rows, dim3(blocks_for((long)n * m)), dim3(256), 0, c.st, Y, W, n, m);
  CTM_HIP(hipGetLastError());
  gemm(c.st, GemmType::F64, n, m, n, 1.0, colmajor(V, n), rowmajor(Y, m), 0.0, out_rowmajor(X, m), 1, c.ws());
  return X;
}

// Rotations 0..3 of A (device, physical frame) into the context's ket and bra copies.
void set_site_tensor(Context& c, int s, const double* A) {
  const long D = c.D, d = c.d;
  DT cur = dt(const_cast<double*>(A), {D, D, D, D, d});
  for (int rot = 0; rot < 4; ++rot) {
    CTM_HIP(hipMemcpyAsync(const_cast<double*>(c.Ak(rot, s)), cur.p, sizeof(double) * c.szk,
                           hipMemcpyDeviceToDevice, c.st));
    CTM_HIP(hipMemcpyAsync(const_cast<double*>(c.Ab(rot, s)), cur.p, sizeof(double) * c.szb,
                           hipMemcpyDeviceToDevice, c.st));
    if (rot < 3) cur = tensor_transpose(c, cur, {1, 2, 3, 0, 4});
  }
}

void fu_bond(Context& c, int s, int dir, const double* g, int als_iters) {
  c.arena.reset();
  const int D = c.D, d = c.d, C = D * d, R3 = D * D * D, r = C, n = r * d, nD = r * D, n2 = r * r;
  const int x = s % c.Lx, y = s / c.Lx;
  const int si = s, li = dir == 0 ? 2 : 1;
  const int sj = dir == 0 ? (x + 1) % c.Lx + c.Lx * y : x + c.Lx * ((y + 1) % c.Ly);
  const int lj = dir == 0 ? 0 : 3;
  const long Dl = D, dl = d;

  // 1. reduced tensors: [k][p][other legs] row-major = column-major R3 x C, QR in place
  DT Ai = dt(const_cast<double*>(c.Ak(0, si)), {Dl, Dl, Dl, Dl, dl});
  DT Aj = dt(const_cast<double*>(c.Ak(0, sj)), {Dl, Dl, Dl, Dl, dl});
  DT Mi = tensor_transpose(c, Ai, {li, 4, other_leg_h(li, 0), other_leg_h(li, 1), other_leg_h(li, 2)});
  DT Mj = tensor_transpose(c, Aj, {lj, 4, other_leg_h(lj, 0), other_leg_h(lj, 1), other_leg_h(lj, 2)});
  double* Ri = c.arena.alloc((size_t)C * C);
  double* Rj = c.arena.alloc((size_t)C * C);
  small_qr(c, Mi.p, R3, C, Ri);
  small_qr(c, Mj.p, R3, C, Rj);

  // 2. bond environment
  double* Ei = c.arena.alloc((size_t)R3 * D * r);
  double* Ej = c.arena.alloc((size_t)R3 * D * r);
  hipLaunchKernelGGL(k_fu_embed, dim3(blocks_for((long)R3 * D * r)), dim3(256), 0, c.st, Mi.p, Ei, D, r, li);
  hipLaunchKernelGGL(k_fu_embed, dim3(blocks_for((long)R3 * D * r)), dim3(256), 0, c.st, Mj.p, Ej, D, r, lj);
  CTM_HIP(hipGetLastError());
  DT Nraw = bond_environment(c, s, dir, Ei, Ej, r);

  // 3. symmetric positive part
  double* V = c.arena.alloc((size_t)n2 * n2);
  double* W = c.arena.alloc(n2);
  double* Vs = c.arena.alloc((size_t)n2 * n2);
  double* Np = c.arena.alloc((size_t)n2 * n2);
  hipLaunchKernelGGL(k_fu_sym, dim3(blocks_for((long)n2 * n2)), dim3(256), 0, c.st, Nraw.p, V, n2);
  CTM_HIP(hipGetLastError());
  sym_eig(c, V, n2, W);
  hipLaunchKernelGGL(k_fu_pos_cols, dim3(blocks_for((long)n2 * n2)), dim3(256), 0, c.st, V, W, Vs, n2);
  CTM_HIP(hipGetLastError());
  gemm(c.st, GemmType::F64, n2, n2, n2, 1.0, colmajor(Vs, n2), rowmajor(V, n2), 0.0, out_rowmajor(Np, n2), 1,
       c.ws());

  // 4. gated core, 5. truncated-SVD start
  double* Th = c.arena.alloc((size_t)n * n);
  double* Tw = c.arena.alloc((size_t)n * n);
  double* S = c.arena.alloc(n);
  double* Ucm = c.arena.alloc((size_t)n * n);
  double* VTcm = c.arena.alloc((size_t)n * n);
  double* bi = c.arena.alloc((size_t)n * D);
  double* bj = c.arena.alloc((size_t)n * D);
  hipLaunchKernelGGL(k_fu_core, dim3(blocks_for((long)n * n)), dim3(256), 0, c.st, Ri, Rj, g, Th, D, d, C);
  CTM_HIP(hipGetLastError());
  CTM_HIP(hipMemcpyAsync(Tw, Th, sizeof(double) * n * n, hipMemcpyDeviceToDevice, c.st));
  la_svd(c.la, Tw, n, S, Ucm, VTcm);
  hipLaunchKernelGGL(k_fu_start, dim3(blocks_for((long)n * D)), dim3(256), 0, c.st, Ucm, VTcm, S, bi, bj, n, D);
  CTM_HIP(hipGetLastError());

  // 6. alternating least squares
  const long rl = r;
  DT N4 = dt(Np, {rl, rl, rl, rl});                      // [x, y, X, Y]
  DT Th4 = dt(Th, {rl, dl, rl, dl});                     // [X, P, Y, Q]
  DT T1 = tensordot(c, N4, {2, 3}, Th4, {0, 2});         // [x, y, P, Q]
  for (int it = 0; it < als_iters; ++it) {
    {
      DT Bj = dt(bj, {rl, dl, Dl});                      // [y, Q, k]
      DT BB = tensordot(c, Bj, {1}, Bj, {1});            // [y, k, Y, K]
      DT Rm = tensor_transpose(c, tensordot(c, N4, {1, 3}, BB, {0, 2}), {0, 2, 1, 3});   // [x, k, X, K]
      DT Sm = tensor_transpose(c, tensordot(c, T1, {1, 3}, Bj, {0, 1}), {0, 2, 1});      // [x, k, P]
      double* X = pinv_solve(c, Rm.p, Sm.p, nD, d);
      bi = tensor_transpose(c, dt(X, {rl, Dl, dl}), {0, 2, 1}).p;                         // [x, P, k]
    }
    {
      DT Bi = dt(bi, {rl, dl, Dl});                      // [x, P, k]
      DT AA = tensordot(c, Bi, {1}, Bi, {1});            // [x, k, X, K]
      DT Rm = tensor_transpose(c, tensordot(c, N4, {0, 2}, AA, {0, 2}), {0, 2, 1, 3});   // [y, k, Y, K]
      DT Sm = tensor_transpose(c, tensordot(c, T1, {0, 2}, Bi, {0, 1}), {0, 2, 1});      // [y, k, Q]
      double* X = pinv_solve(c, Rm.p, Sm.p, nD, d);
      bj = tensor_transpose(c, dt(X, {rl, Dl, dl}), {0, 2, 1}).p;                         // [y, Q, k]
    }
  }

  // 7. A' = X b back to [l][u][r][d][p], sign rule, normalisation
  double* Oi = c.arena.alloc((size_t)R3 * d * D);
  double* Oj = c.arena.alloc((size_t)R3 * d * D);
  gemm(c.st, GemmType::F64, R3, d * D, r, 1.0, colmajor(Mi.p, R3), rowmajor(bi, d * D), 0.0,
       out_rowmajor(Oi, d * D), 1, c.ws());
  gemm(c.st, GemmType::F64, R3, d * D, r, 1.0, colmajor(Mj.p, R3), rowmajor(bj, d * D), 0.0,
       out_rowmajor(Oj, d * D), 1, c.ws());
  auto back = [&](int leg) {
    std::vector<int> perm(5);
    int t = 0;
    for (int L = 0; L < 4; ++L) perm[L] = (L == leg) ? 4 : t++;
    perm[4] = 3;
    return perm;
  };
  DT Ani = tensor_transpose(c, dt(Oi, {Dl, Dl, Dl, dl, Dl}), back(li));   // [o1 o2 o3 P k] -> [l u r d p]
  DT Anj = tensor_transpose(c, dt(Oj, {Dl, Dl, Dl, dl, Dl}), back(lj));
  hipLaunchKernelGGL(k_fu_sign_normalize, dim3(1), dim3(256), 0, c.st, Ani.p, Anj.p, D, d, li, lj);
  CTM_HIP(hipGetLastError());
  set_site_tensor(c, si, Ani.p);
  set_site_tensor(c, sj, Anj.p);
}

}  // namespace

void full_update_step(Context& c, const double* H, double tau, int als_iters, int env_sweeps) {
  CTM_CHECK(c.layers == 2 && c.R == 1 && c.ctype == GemmType::F64, -1,
            "the full update needs an FP64 iTPS context of one solve");
  CTM_CHECK(c.Lx >= 2 && c.Ly >= 2, -1, "the full update needs Lx >= 2 and Ly >= 2");
  CTM_CHECK(c.D * c.D >= c.d && c.DK == c.D && c.DB == c.D, -1, "the full update needs d <= D^2");
  const int N = c.N, d2 = c.d * c.d;
  for (long e = 0; e < (long)N * 2 * d2 * d2; ++e) CTM_CHECK(std::isfinite(H[e]), -1, "Hamiltonian entries must be finite");
  CTM_CHECK(std::isfinite(tau) && tau >= 0.0, -1, "tau must be finite and >= 0");
  DevBuf Hd, taud, gates;
  Hd.alloc(sizeof(double) * N * 2 * d2 * d2);
  taud.alloc(sizeof(double));
  gates.alloc(sizeof(double) * N * 2 * d2 * d2);
  CTM_HIP(hipMemcpyAsync(Hd.p, H, Hd.bytes, hipMemcpyHostToDevice, c.st));
  CTM_HIP(hipMemcpyAsync(taud.p, &tau, sizeof(double), hipMemcpyHostToDevice, c.st));
  trotter_gates(c.st, Hd.as<double>(), taud.as<double>(), gates.as<double>(), N, d2, 1);
  for (int dir = 0; dir < 2; ++dir)
    for (int s = 0; s < N; ++s) {
      fu_bond(c, s, dir, gates.as<double>() + (long)(s * 2 + dir) * d2 * d2, als_iters);
      if (env_sweeps > 0) {
        int done = 0, conv = 0;
        double delta = 0.0;
        do_sweeps(c, env_sweeps, 0.0, &done, &delta, &conv);
      }
    }
  CTM_HIP(hipStreamSynchronize(c.st));
}

void get_site_tensors(Context& c, double* out) {
  for (int s = 0; s < c.N; ++s)
    CTM_HIP(hipMemcpyAsync(out + (long)s * c.szk, c.Ak(0, s), sizeof(double) * c.szk, hipMemcpyDeviceToHost, c.st));
  CTM_HIP(hipStreamSynchronize(c.st));
}

}  // namespace ctm
