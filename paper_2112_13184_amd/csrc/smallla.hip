// FP64 factorisations of the projector computation, written for one MI355X.
//
// * Cholesky QR of a tall n x k panel Y: G = Y^T Y (MFMA GEMM), G (+ shift) =
//   L L^T in one 1024-thread workgroup with the matrix in registers, 2-D
//   cyclic over a 32 x 32 thread grid (outer-product form, one barrier per
//   column), R^-1 = L^-T one wave per
//   column, then Y <- Y R^-1 (MFMA GEMM).  The first pass uses the shift of
//   Fukaya, Kannan, Nakatsukasa, Yamamoto and Yanagisawa (SIAM J. Sci. Comput.
//   42 (2020) A477), s = 11 (n k + k (k + 1)) u ||Y||_F^2, which keeps the Gram
//   matrix positive definite for condition numbers up to about 1e12; two more
//   unshifted passes restore orthogonality to working precision.
// * SVD of a k x k matrix by block one-sided Jacobi (Hestenes): the columns are
//   split into an even number of blocks; each kernel launch orthogonalises the
//   column pairs inside every block pair of one round of a round-robin
//   tournament, with the two blocks and their rotation accumulators staged in
//   LDS.  A sweep is one full tournament; sweeps stop on the device once no
//   pair is rotated by more than the tolerance.
#include "smallla.hpp"
#include "wave.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace ctm {
namespace {

constexpr int kCholThreads = 1024;
constexpr int kCholT = 32;                                       // threads as a kCholT x kCholT grid
// row / column blocks per thread: 6 up to k = 192, 10 up to k = 320 (the
// larger form keeps 55 blocks per thread and spills part of them)
constexpr int kCholBSmall = 6;
constexpr int kCholBLarge = (kSmallLAMaxK + kCholT - 1) / kCholT;
static_assert(kCholT * kCholT == kCholThreads, "k_chol: thread grid");
// Jacobi: columns per block (one wave per pair of a round, 16 blocks at k = 192)
constexpr int kJacobiMaxBS = 12;
// rows per lane of the triangular inverse and the Jacobi rounds: 3 up to
// k = 192, 5 up to k = 320
constexpr int kRowsSmall = 3;
constexpr int kRowsLarge = (kSmallLAMaxK + 63) / 64;
// failure code of a problem whose Jacobi SVD did not converge (Cholesky
// failures use 10 * pass + 1 or 2)
constexpr int kJacobiUnconverged = 100;


__device__ double block_reduce(double v, bool is_max, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = is_max ? wave_max(v) : wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = is_max ? fmax(r, sh[i]) : r + sh[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int tri(int i, int l) { return i * (i + 1) / 2 + l; }

// Register blocks of one k_chol thread: row block a, column block c, a >= c.
template <int KB> struct CholBlocks { static constexpr int NB = KB * (KB + 1) / 2; };
__host__ __device__ constexpr int cblk(int a, int c) { return a * (a + 1) / 2 + c; }

// Column j (in column block JB) -> LDS, by the threads that hold it, with
// the rows at and above the pivot taken as zero so that the update needs no
// masks of its own; the thread holding the pivot also stores it and its
// reciprocal (computed once per step instead of once per thread).
template <int KB, int JB>
__device__ __forceinline__ void chol_publish(const double (&val)[CholBlocks<KB>::NB], double* cj, int tx, int j,
                                             double* pv, double* iv) {
#pragma unroll
  for (int a = JB; a < KB; ++a) {
    const int i = tx + kCholT * a;
    cj[i] = (i > j) ? val[cblk(a, JB)] : 0.0;
  }
  if (tx == j % kCholT) {
    const double d = val[cblk(JB, JB)];
    *pv = d;
    *iv = 1.0 / d;
  }
}

// Rank-one update by the pivot column j (in column block JB): the published
// column is zero at and above the pivot and outside k x k, so entries right
// of and below the pivot lose fi * fl and all others lose exactly zero.
// Blocks left of JB are finished and not touched.
template <int KB, int JB>
__device__ __forceinline__ void chol_update(double (&val)[CholBlocks<KB>::NB], const double* cj, double inv, int tx,
                                            int ty) {
  double fl[KB], fi[KB];
#pragma unroll
  for (int c = JB; c < KB; ++c) {
    fl[c] = cj[ty + kCholT * c] * inv;
    fi[c] = cj[tx + kCholT * c];
  }
#pragma unroll
  for (int a = JB; a < KB; ++a)
#pragma unroll
    for (int c = JB; c <= a; ++c) val[cblk(a, c)] -= fi[a] * fl[c];
}

// G_b (k x k, col-major) [+ s I] = L L^T, rank revealing: a pivot below
// drop_rel times the largest one so far marks its column as dependent
// (mask 0): the column is taken as zero and R = L^T, the output, gets a zero
// row there (so that accumulated factors keep the zero); the triangular
// inverse takes a unit diagonal in its place.  shifted: add s = shift_scale
// * trace(G).
// check_id: flag the problem if the non-zero part of G is not within 0.5 of
// the identity.  NaN / Inf pivots flag the problem too.
// The lower triangle lives in registers, distributed 2-D cyclically: thread
// (ty, tx) of the 32 x 32 grid holds rows tx + 32 a and columns ty + 32 c
// for the 21 block pairs a >= c.  Step j broadcasts column j through a
// double-buffered LDS column (one barrier per step); the update is
// specialised on the block of j, so finished blocks cost nothing.  R is
// written through an LDS tile, 32 rows of L at a time, so that it is stored
// along contiguous columns.
template <int KB>
__global__ __launch_bounds__(kCholThreads) void k_chol(const double* G, int k, int pass, int shifted,
                                                        int check_id, double shift_scale, double drop_rel,
                                                        double* Rout, double* mask, int* flag) {
  constexpr int NB = CholBlocks<KB>::NB;
  __shared__ double col[2][KB * kCholT];
  __shared__ double pv[2], iv[2];
  __shared__ double tile[kCholT][KB * kCholT + 1];
  __shared__ double piv[KB * kCholT];
  __shared__ double red[16];
  __shared__ int bad;
  __shared__ unsigned char dropped[KB * kCholT];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int tx = tid % kCholT, ty = tid / kCholT;
  const long kk2 = (long)k * k;
  const double* g = G + b * kk2;
  if (tid == 0) bad = 0;
  double tr = 0.0;
  for (int i = tid; i < k; i += blockDim.x) tr += g[i + (long)i * k];
  tr = block_reduce(tr, false, red);
  const double s = shifted ? shift_scale * tr : 0.0;
  // val[cblk(a, c)] = entry (row tx + 32 a, column ty + 32 c); entries above
  // the diagonal or outside k x k start at zero and are never output
  double val[NB];
  double dev = 0.0;
#pragma unroll
  for (int a = 0; a < KB; ++a)
#pragma unroll
    for (int c = 0; c <= a; ++c) {
      const int i = tx + kCholT * a, l = ty + kCholT * c;
      double v = 0.0;
      if (i < k && l <= i) {
        v = g[i + (long)l * k];
        if (check_id) {
          const double gi = g[i + (long)i * k], gl = g[l + (long)l * k];
          if (gi > 1e-3 && gl > 1e-3) dev = fmax(dev, fabs(v - (i == l ? 1.0 : 0.0)));
        }
        if (i == l) v += s;
      }
      val[cblk(a, c)] = v;
    }
  if (check_id) {
    dev = block_reduce(dev, true, red);
    if (tid == 0 && !(dev <= 0.5)) bad = 2;
  }
  double dmax = 0.0;
  for (int j = 0; j < k; ++j) {
    double* cj = col[j & 1];
    const int jb = j / kCholT;
    if (ty == j % kCholT) {
      switch (jb) {
#define CHOL_PUBLISH(J) \
  case J:                \
    if constexpr (J < KB) chol_publish<KB, J>(val, cj, tx, j, &pv[j & 1], &iv[j & 1]); \
    break;
        CHOL_PUBLISH(0) CHOL_PUBLISH(1) CHOL_PUBLISH(2) CHOL_PUBLISH(3) CHOL_PUBLISH(4)
        CHOL_PUBLISH(5) CHOL_PUBLISH(6) CHOL_PUBLISH(7) CHOL_PUBLISH(8) CHOL_PUBLISH(9)
#undef CHOL_PUBLISH
      }
    }
    __syncthreads();
    const double d = pv[j & 1];
    const bool drop = !(d > drop_rel * dmax) || !(d > 0.0) || !isfinite(d);
    if (tid == 0) {
      dropped[j] = drop ? 1 : 0;
      piv[j] = d;
      if (!isfinite(d)) bad = 1;
    }
    if (!drop) {
      dmax = fmax(dmax, d);
      const double inv = iv[j & 1];
      switch (jb) {
#define CHOL_UPDATE(J) \
  case J:               \
    if constexpr (J < KB) chol_update<KB, J>(val, cj, inv, tx, ty); \
    break;
        CHOL_UPDATE(0) CHOL_UPDATE(1) CHOL_UPDATE(2) CHOL_UPDATE(3) CHOL_UPDATE(4)
        CHOL_UPDATE(5) CHOL_UPDATE(6) CHOL_UPDATE(7) CHOL_UPDATE(8) CHOL_UPDATE(9)
#undef CHOL_UPDATE
      }
    }
  }
  __syncthreads();
  double* Rb = Rout + b * kk2;
  // scale factors of this thread's columns
  double sd[KB];
  bool dr[KB];
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    const int l = ty + kCholT * c;
    dr[c] = l < k ? dropped[l] != 0 : true;
    sd[c] = (l < k && !dr[c]) ? sqrt(piv[l]) : 1.0;
  }
  // R = L^T with zero rows where dropped: rows 32 a .. 32 a + 31 of L go
  // through the tile and out as columns of R
#pragma unroll
  for (int a = 0; a < KB; ++a) {
    const int i = tx + kCholT * a;
#pragma unroll
    for (int c = 0; c < KB; ++c) {
      const int l = ty + kCholT * c;
      double r = 0.0;
      if (c <= a && i < k && l <= i && !dr[c]) r = (i == l) ? sd[c] : val[cblk(a, c)] / sd[c];
      tile[tx][l] = r;
    }
    __syncthreads();
    const int ri = kCholT * a + ty;        // column of R = row of L
    if (ri < k) {
#pragma unroll
      for (int m = 0; m < KB; ++m) {
        const int l = tx + kCholT * m;
        if (l < k) Rb[l + (long)ri * k] = tile[ty][l];   // R[l][ri] = L[ri][l]
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < k; j += blockDim.x) mask[(long)b * k + j] = dropped[j] ? 0.0 : 1.0;
  // reason code: 10 * pass + 1 (non-finite pivot) or + 2 (not orthonormal)
  if (tid == 0 && bad) flag[b] = max(flag[b], 10 * pass + bad);
}

// Rinv = U^-1 for the upper triangular U = L^T, one wave per column c.  U
// equals the stored R except on the diagonal of dropped directions, where
// R has zero rows and U a unit diagonal (mask 0).  Column c of U^-1 solves
// U x = e_c by back substitution in column form: from row c up, x_i = b_i /
// U[i][i], then b loses x_i times column i of U.  A step thus waits on one
// lane broadcast, not on a wave reduction.  Column i of R does not depend on
// the solution, so the columns of the next 16 steps are kept in flight in a
// register ring.  The update also touches row i (and rows below it, where R
// is zero); x_i is kept apart, so that does not matter.
template <int ROWS>
__global__ __launch_bounds__(256) void k_trinv(const double* R, const double* mask, int k, double* Rinv) {
  constexpr int RING = 16;
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (c >= k) return;
  const long kk2 = (long)k * k;
  const double* Rb = R + b * kk2;
  const double* mb = mask + (long)b * k;
  double bv[ROWS], rd[ROWS], xo[ROWS];        // rows lane + 64 q: right-hand side, 1 / U[i][i], solution
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    const int i = lane + 64 * q;
    bv[q] = (i == c) ? 1.0 : 0.0;
    xo[q] = 0.0;
    rd[q] = (i <= c) ? (mb[i] != 0.0 ? 1.0 / Rb[i + (long)i * k] : 1.0) : 0.0;
  }
  double ring[RING][ROWS];
  auto fetch = [&](int i, double* dst) {
    const long col = (long)(i < 0 ? 0 : i) * k;
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
      const int kx = lane + 64 * q;
      dst[q] = Rb[(kx < k ? kx : k - 1) + col];                  // R[kx][i]
    }
  };
#pragma unroll
  for (int s = 0; s < RING; ++s) fetch(c - s, ring[s]);
  for (int base = c; base >= 0; base -= RING) {
#pragma unroll
    for (int s = 0; s < RING; ++s) {
      const int i = base - s;
      if (i < 0) break;
      double col[ROWS];
#pragma unroll
      for (int q = 0; q < ROWS; ++q) col[q] = ring[s][q];
      fetch(i - RING, ring[s]);
      const int qi = i >> 6, li = i & 63;
      double bq = bv[0], rq = rd[0];
#pragma unroll
      for (int q = 1; q < ROWS; ++q) {
        bq = (qi == q) ? bv[q] : bq;
        rq = (qi == q) ? rd[q] : rq;
      }
      const double xi = readlane_f64(bq * rq, li);
#pragma unroll
      for (int q = 0; q < ROWS; ++q) {
        xo[q] = (q == qi && lane == li) ? xi : xo[q];
        bv[q] = fma(-xi, col[q], bv[q]);
      }
    }
  }
  // a dropped direction c gets a zero column, so that Y U^-1 has a zero
  // column there (the product applies the mask)
  const bool keep = mb[c] != 0.0;
  double* out = Rinv + b * kk2 + (long)c * k;
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    const int i = lane + 64 * q;
    if (i < k) out[i] = (keep && i <= c) ? xo[q] : 0.0;
  }
}

// dst_b = src_b with column j scaled by mask_b[j] (column-major n x k panels;
// mask null: a plain copy).
__global__ void k_copy_panels(const double* src, long sstride, double* dst, long dstride, int n, int k,
                              const double* mask) {
  const int b = blockIdx.y;
  const long elems = (long)n * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < elems; e += (long)gridDim.x * blockDim.x)
    dst[b * dstride + e] = mask ? src[b * sstride + e] * mask[(long)b * k + e / n] : src[b * sstride + e];
}

// ---------------------------------------------------------------------------
// block one-sided Jacobi
// ---------------------------------------------------------------------------
__global__ void k_jacobi_init(double* J, int k, double* off, int* conv, int* nsweep) {
  const int b = blockIdx.y;
  const long kk2 = (long)k * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < kk2; e += (long)gridDim.x * blockDim.x)
    J[b * kk2 + e] = ((e % k) == (e / k)) ? 1.0 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    off[b] = 0.0;
    conv[b] = 0;
    nsweep[b] = 0;
  }
}

// Per-problem convergence state of a value-only Jacobi (no rotation matrix).
__global__ void k_jacobi_init_values(double* off, int* conv, int* nsweep, int batch) {
  const int b = threadIdx.x;
  if (b < batch) {
    off[b] = 0.0;
    conv[b] = 0;
    nsweep[b] = 0;
  }
}

// S_b = the column norms of the rotated A_b (its singular values), in
// descending order (ties by column index): one workgroup per problem, k <= 320.
__global__ __launch_bounds__(256) void k_colnorm_desc(const double* A, int k, double* S, long sstride) {
  __shared__ double nrm[kSmallLAMaxK];
  const int b = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* Ab = A + (long)b * k * k;
  for (int col = w; col < k; col += blockDim.x >> 6) {
    double s2 = 0.0;
    for (int r = lane; r < k; r += 64) {
      const double v = Ab[(long)col * k + r];
      s2 += v * v;
    }
    s2 = wave_sum(s2);
    if (lane == 0) nrm[col] = sqrt(s2);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double v = nrm[i];
    int rank = 0;
    for (int j = 0; j < k; ++j) rank += (nrm[j] > v) || (nrm[j] == v && j < i);
    S[(long)b * sstride + rank] = v;
  }
}

// After a sweep: converged if no pair needed a rotation (off = 0); nsweep
// counts the sweeps that ran.
// Problems whose Jacobi SVD has not converged get a failure code in the
// Cholesky-failure slots, so that their cuts take the Householder path.
__global__ void k_jacobi_mark_unconverged(const int* conv, int* fail, int batch) {
  const int b = threadIdx.x;
  if (b < batch && !conv[b]) fail[b] = max(fail[b], kJacobiUnconverged);
}

// Cyclic Jacobi converges quadratically: after a sweep whose rotated pairs
// all had |ga| / sqrt(al be) <= stop, the next sweep's would be of order
// stop^2, below the rotation threshold for the stops used here, so the
// problem is done without running that (rotation-free) check sweep.
__global__ void k_jacobi_sweep_end(double* off, int* conv, int* nsweep, int batch, double stop) {
  const int b = threadIdx.x;
  if (b < batch) {
    if (!conv[b]) ++nsweep[b];
    if (off[b] <= stop) conv[b] = 1;
    off[b] = 0.0;
  }
}

__device__ __forceinline__ int circle(int pos, int round, int m) {
  // position pos in round `round` (< m - 1) of a round-robin tournament of m
  // (even) players, pos < m
  if (pos == 0) return 0;
  int t = pos - 1 + round;
  if (t >= m - 1) t -= m - 1;
  return t + 1;
}

// 1 / sqrt(x) for normal or subnormal x > 0: the hardware estimate (about 23
// correct bits) and two Newton steps y += y (1 - x y^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double h = x * y;
    const double e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Rotation of the column pair (x, y) with accumulators (u, v), held by one
// wave (rows lane + 64 t): rotate when |ga| > tol sqrt(al be); the angle
// zeroing the inner product has tan(2 theta) = 2 ga / (be - al), and with
// d = be - al, r = sqrt(d^2 + 4 ga^2), w = sqrt(2 r (r + |d|)) its cosine and
// sine are (r + |d|) / w and 2 ga sgn(d) / w: two reciprocal square roots.
// Returns |ga| / sqrt(al be) of a rotated pair, else 0 (uniform over the wave).
template <int ROWS, bool VEC>
__device__ __forceinline__ double jacobi_pair(double (&x)[ROWS], double (&y)[ROWS], double (&u)[ROWS],
                                              double (&v)[ROWS], double tol) {
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int t = 0; t < ROWS; ++t) {
    al += x[t] * x[t];
    be += y[t] * y[t];
    ga += x[t] * y[t];
  }
  al = wave_sum(al);
  be = wave_sum(be);
  ga = wave_sum(ga);
  const double ab = al * be, g2 = ga * ga;
  if (!(g2 > tol * tol * ab)) return 0.0;
  const double dd = be - al, ad = fabs(dd);
  const double X = dd * dd + 4.0 * g2;
  const double r = X * rsqrt_nr(X);
  const double inv = rsqrt_nr(2.0 * r * (r + ad));
  const double cs = (r + ad) * inv, sn = 2.0 * ga * (dd >= 0.0 ? inv : -inv);
#pragma unroll
  for (int t = 0; t < ROWS; ++t) {
    const double xn = cs * x[t] - sn * y[t], yn = sn * x[t] + cs * y[t];
    x[t] = xn;
    y[t] = yn;
    if (VEC) {
      const double un = cs * u[t] - sn * v[t], vn = sn * u[t] + cs * v[t];
      u[t] = un;
      v[t] = vn;
    }
  }
  return fabs(ga) * rsqrt_nr(ab);
}

// One tournament round over blocks: workgroup w of problem b orthogonalises
// column pairs of its block pair (columns >= k are zero padding), one wave
// per column pair of each inner step (launched with 64 * bs threads).  In
// round 0 every block meets another one, so that round runs the full
// tournament of the 2 bs columns (the pairs inside each block and across),
// all staged in LDS.  Later rounds take only the bs^2 pairs across the two
// blocks, in bs steps of bs disjoint pairs: wave q pairs column q of the
// first block, which it keeps in registers for the whole round, with the
// columns of the second block in turn, so that a step moves only those
// through LDS (the LDS traffic of a step bounds its time).  Each column pair
// is rotated once per sweep.  off[b] receives the largest |ga| / sqrt(al be)
// of the pairs rotated (positive doubles order like their bits).
// VEC = false: singular values only (J is not touched).
template <int ROWS, bool VEC = true>
__global__ __launch_bounds__(64 * kJacobiMaxBS) void k_jacobi_round(double* A, double* J, int k, int nb, int bs,
                                                                   int round, double* off, const int* conv,
                                                                   double tol) {
  // staged columns are kJacobiLd apart and zero past row k, so that the
  // steps read and write whole columns without row checks
  constexpr int kJacobiLd = 64 * ROWS;
  __shared__ double sA[2 * kJacobiMaxBS * kJacobiLd];
  __shared__ double sJ[VEC ? 2 * kJacobiMaxBS * kJacobiLd : 1];
  const int b = blockIdx.y;
  if (conv[b]) return;
  const long kk2 = (long)k * k;
  double* Ab = A + b * kk2;
  double* Jb = J + b * kk2;
  const int pa = circle(blockIdx.x, round, nb), pb = circle(nb - 1 - blockIdx.x, round, nb);
  const int m = 2 * bs;
  // the wave index is uniform: keep it (and the column arithmetic) scalar
  const int lane = threadIdx.x & 63, q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gcol[2] = {pa * bs + q, pb * bs + q};
  // wave q loads local columns q (block pa) and bs + q (block pb): all global
  // loads first, then the LDS stores (column q of pa stays in registers after
  // round 0)
  double x[ROWS], u[ROWS];
  {
    double va[2][ROWS], vj[2][ROWS];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int t = 0; t < ROWS; ++t) {
        const int r = lane + 64 * t;
        const bool ok = gcol[h] < k && r < k;
        va[h][t] = ok ? Ab[(long)gcol[h] * k + r] : 0.0;
        vj[h][t] = (VEC && ok) ? Jb[(long)gcol[h] * k + r] : 0.0;
      }
#pragma unroll
    for (int t = 0; t < ROWS; ++t) {
      x[t] = va[0][t];
      u[t] = vj[0][t];
    }
#pragma unroll
    for (int h = (round == 0 ? 0 : 1); h < 2; ++h)
#pragma unroll
      for (int t = 0; t < ROWS; ++t) {
        const int r = lane + 64 * t;
        sA[(h * bs + q) * kJacobiLd + r] = va[h][t];
        if (VEC) sJ[(h * bs + q) * kJacobiLd + r] = vj[h][t];
      }
  }
  __syncthreads();
  double offl = 0.0;
  if (round == 0) {
    for (int st = 0; st < m - 1; ++st) {
      const int ci = circle(q, st, m), cj = circle(m - 1 - q, st, m);
      double* ai = sA + ci * kJacobiLd + lane;
      double* aj = sA + cj * kJacobiLd + lane;
      double* ji = sJ + (VEC ? ci * kJacobiLd + lane : 0);
      double* jj = sJ + (VEC ? cj * kJacobiLd + lane : 0);
      double xa[ROWS], ya[ROWS], ua[ROWS], vb[ROWS];
#pragma unroll
      for (int t = 0; t < ROWS; ++t) {
        xa[t] = ai[64 * t];
        ya[t] = aj[64 * t];
        ua[t] = VEC ? ji[64 * t] : 0.0;
        vb[t] = VEC ? jj[64 * t] : 0.0;
      }
      const double mu = jacobi_pair<ROWS, VEC>(xa, ya, ua, vb, tol);
      if (mu > 0.0) {
        offl = fmax(offl, mu);
#pragma unroll
        for (int t = 0; t < ROWS; ++t) {
          ai[64 * t] = xa[t];
          aj[64 * t] = ya[t];
          if (VEC) {
            ji[64 * t] = ua[t];
            jj[64 * t] = vb[t];
          }
        }
      }
      __syncthreads();
    }
  } else {
    int cl = q;                                      // (q + st) mod bs
    for (int st = 0; st < bs; ++st) {
      double* aj = sA + (bs + cl) * kJacobiLd + lane;
      double* jj = sJ + (VEC ? (bs + cl) * kJacobiLd + lane : 0);
      cl = (cl + 1 == bs) ? 0 : cl + 1;
      double y[ROWS], v[ROWS];
#pragma unroll
      for (int t = 0; t < ROWS; ++t) {
        y[t] = aj[64 * t];
        v[t] = VEC ? jj[64 * t] : 0.0;
      }
      const double mu = jacobi_pair<ROWS, VEC>(x, y, u, v, tol);
      if (mu > 0.0) {
        offl = fmax(offl, mu);
#pragma unroll
        for (int t = 0; t < ROWS; ++t) {
          aj[64 * t] = y[t];
          if (VEC) jj[64 * t] = v[t];
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int gc = gcol[h];
    if (gc < k) {
#pragma unroll
      for (int t = 0; t < ROWS; ++t) {
        const int r = lane + 64 * t;
        if (r < k) {
          const bool reg = (h == 0 && round > 0);
          Ab[(long)gc * k + r] = reg ? x[t] : sA[(h * bs + q) * kJacobiLd + r];
          if (VEC) Jb[(long)gc * k + r] = reg ? u[t] : sJ[(h * bs + q) * kJacobiLd + r];
        }
      }
    }
  }
  __shared__ double red[kJacobiMaxBS];
  offl = wave_max(offl);
  if (lane == 0) red[q] = offl;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = red[0];
    for (int i = 1; i < bs; ++i) mx = fmax(mx, red[i]);
    atomicMax(reinterpret_cast<unsigned long long*>(off + b), (unsigned long long)__double_as_longlong(mx));
  }
}

// Sum over each half (32 lanes) of the wave; every lane of a half receives
// its half's sum.  DPP inside the rows of 16, then row 0 into row 1 and row 2
// into row 3 (row_bcast:15), read from lanes 31 and 63.
__device__ __forceinline__ double half_sum(double v, bool upper) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  v += dpp_rows_f64<0x142, 0xA>(0.0, v);
  const double lo = readlane_f64(v, 31), hi = readlane_f64(v, 63);
  return upper ? hi : lo;
}

// One-sided Jacobi of one small m x m matrix per workgroup, the whole matrix
// in LDS (column stride LD, rows past m zero) and every sweep in the one
// launch: cyclic tournament over the columns (padded to an even count with a
// zero column), one half-wave (32 lanes, LD / 32 rows each) per column pair
// of a round, so that the sixteen waves take 32 pairs at once; the same
// rotation and threshold as the blocked Jacobi, and no rotation of columns at
// the rounding level of the matrix.  Stops after a sweep without
// rotations, after a sweep whose largest rotated |ga| / sqrt(al be) was at
// most `stop` (the next sweep's would be of order stop^2, below tol for
// stop = 1e-10; stop = 0: only the first rule), or after max_sweeps.
// VEC = false (m <= 128): S_b (m values, descending) = the column norms.
// VEC = true (m <= 64): the rotations are also accumulated in J (from the
// identity); A_b and J_b are written back (column-major, ld m) for the
// finishing kernel, as after the blocked Jacobi.
template <int LD, bool VEC>
__global__ __launch_bounds__(1024) void k_jacobi_onewg(double* A, int m, double* S, double* J, double tol,
                                                       double stop, int max_sweeps, int* fail) {
  constexpr int NCOL = LD;                       // columns held (m rounded up to even <= LD)
  __shared__ double sA[NCOL * LD];
  __shared__ double sJ[VEC ? NCOL * LD : 1];
  __shared__ double sig[NCOL];
  __shared__ int rotated;
  __shared__ unsigned long long offmax;          // largest rotated ratio of the sweep (bits)
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), nw = blockDim.x >> 6;
  const bool upper = lane >= 32;
  const int hl = lane & 31;
  const int m2 = m + (m & 1);
  double* Ab = A + (long)b * m * m;
  for (int e = tid; e < m2 * LD; e += blockDim.x) {
    const int col = e / LD, r = e % LD;
    sA[e] = (col < m && r < m) ? Ab[(long)col * m + r] : 0.0;
    if (VEC) sJ[e] = (col == r && col < m) ? 1.0 : 0.0;
  }
  constexpr int RW = LD / 32;                    // rows per lane
  // columns with |c|^2 <= 1e-30 ||A||_F^2 are at the rounding level of the
  // matrix: pairs with such a column are not rotated (noise columns would
  // otherwise keep rotating against each other at O(1) angles)
  __shared__ double fred[16];
  double f2 = 0.0;
  __syncthreads();
  for (int e = tid; e < m2 * LD; e += blockDim.x) f2 += sA[e] * sA[e];
  f2 = wave_sum(f2);
  if (lane == 0) fred[w] = f2;
  __syncthreads();
  double fro2 = 0.0;
  for (int i = 0; i < nw; ++i) fro2 += fred[i];
  const double tiny = 1e-30 * fro2;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (tid == 0) {
      rotated = 0;
      offmax = 0ull;
    }
    __syncthreads();
    for (int round = 0; round < m2 - 1; ++round) {
      // pair slots: half h of wave w takes pairs 2 w + h, 2 w + h + 2 nw, ...
      for (int q0 = 2 * w; q0 < m2 / 2; q0 += 2 * nw) {
        const int q = q0 + (upper ? 1 : 0);
        const bool act = q < m2 / 2;
        const int ci = act ? circle(q, round, m2) : 0, cj = act ? circle(m2 - 1 - q, round, m2) : 0;
        double* ai = sA + ci * LD + hl;
        double* aj = sA + cj * LD + hl;
        double x[RW], y[RW];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int t = 0; t < RW; ++t) {
          x[t] = act ? ai[32 * t] : 0.0;
          y[t] = act ? aj[32 * t] : 0.0;
          al += x[t] * x[t];
          be += y[t] * y[t];
          ga += x[t] * y[t];
        }
        al = half_sum(al, upper);
        be = half_sum(be, upper);
        ga = half_sum(ga, upper);
        const double ab = al * be, g2 = ga * ga;
        if (act && al > tiny && be > tiny && g2 > tol * tol * ab) {
          const double dd = be - al, ad = fabs(dd);
          const double X = dd * dd + 4.0 * g2;
          const double r = X * rsqrt_nr(X);
          const double inv = rsqrt_nr(2.0 * r * (r + ad));
          const double cs = (r + ad) * inv, sn = 2.0 * ga * (dd >= 0.0 ? inv : -inv);
#pragma unroll
          for (int t = 0; t < RW; ++t) {
            ai[32 * t] = cs * x[t] - sn * y[t];
            aj[32 * t] = sn * x[t] + cs * y[t];
          }
          if (VEC) {
            double* ji = sJ + ci * LD + hl;
            double* jj = sJ + cj * LD + hl;
#pragma unroll
            for (int t = 0; t < RW; ++t) {
              const double u = ji[32 * t], v = jj[32 * t];
              ji[32 * t] = cs * u - sn * v;
              jj[32 * t] = sn * u + cs * v;
            }
          }
          if (hl == 0) {
            rotated = 1;
            const double ratio = fabs(ga) * rsqrt_nr(ab);
            atomicMax(&offmax, (unsigned long long)__double_as_longlong(ratio));
          }
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    const double worst = __longlong_as_double((long long)offmax);
    __syncthreads();
    if (!any || worst <= stop) break;
    // still rotating after the last allowed sweep: not converged
    if (sw == max_sweeps - 1 && fail && tid == 0) fail[b] = max(fail[b], kJacobiUnconverged);
  }
  if (VEC) {
    double* Jb = J + (long)b * m * m;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int col = e / m, r = e % m;
      Ab[e] = sA[col * LD + r];
      Jb[e] = sJ[col * LD + r];
    }
    return;
  }
  for (int col = w; col < m; col += nw) {
    double s2 = 0.0;
#pragma unroll
    for (int t = 0; t < LD / 64; ++t) {
      const double v = sA[col * LD + lane + 64 * t];
      s2 += v * v;
    }
    s2 = wave_sum(s2);
    if (lane == 0) sig[col] = sqrt(s2);
  }
  __syncthreads();
  for (int col = tid; col < m; col += blockDim.x) {
    int rnk = 0;
    for (int o = 0; o < m; ++o) rnk += (sig[o] > sig[col]) || (sig[o] == sig[col] && o < col);
    S[(long)b * m + rnk] = sig[col];
  }
}

constexpr int kJacobiOneWgMaxK = 64;   // SVD with vectors in one workgroup up to this k

// Column norms -> singular values, sorted descending; X = A S^-1, Y = J.
__global__ __launch_bounds__(256) void k_svd_finalize(const double* A, const double* J, int k, double* X,
                                                       double* S, long sstride, double* Y) {
  __shared__ double sig[kSmallLAMaxK];
  __shared__ int pos[kSmallLAMaxK];
  const int b = blockIdx.x;
  const long kk2 = (long)k * k;
  const double* Ab = A + b * kk2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wv; c < k; c += nw) {
    double s = 0.0;
    for (int r = lane; r < k; r += 64) s += Ab[(long)c * k + r] * Ab[(long)c * k + r];
    s = wave_sum(s);
    if (lane == 0) sig[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    int rnk = 0;
    for (int o = 0; o < k; ++o) rnk += (sig[o] > sig[c]) || (sig[o] == sig[c] && o < c);
    pos[c] = rnk;
  }
  __syncthreads();
  for (long e = threadIdx.x; e < kk2; e += blockDim.x) {
    const int r = (int)(e % k), c = (int)(e / k);
    const int p = pos[c];
    const double sc = sig[c];
    X[b * kk2 + (long)p * k + r] = (sc > 0.0) ? Ab[e] / sc : 0.0;
    Y[b * kk2 + (long)p * k + r] = J[b * kk2 + e];
  }
  for (int c = threadIdx.x; c < k; c += blockDim.x) S[(long)b * sstride + pos[c]] = sig[c];
}


}  // namespace

void smallla_alloc(SmallLA& s, int kmax, int batch_max, long nmax) {
  s.kmax = kmax;
  s.batch_max = batch_max;
  const size_t m = (size_t)kmax * kmax * batch_max;
  s.G.alloc(m * 8); s.R.alloc(m * 8); s.Rinv.alloc(m * 8);
  s.Racc.alloc(m * 8); s.Rtmp.alloc(m * 8); s.J.alloc(m * 8);
  CTM_CHECK(batch_max <= 64, -1, "smallla: at most 64 problems per batch");
  s.flag.alloc(sizeof(int) * 256);
  s.hflag.alloc(sizeof(int) * 256);
  s.off.alloc(sizeof(double) * 64);
  s.mask.alloc(sizeof(double) * (size_t)kmax * batch_max);
  s.tmp_elems = (size_t)nmax * kmax * batch_max;
  s.tmp.alloc(s.tmp_elems * 8);
  CTM_HIP(hipMemset(s.flag.p, 0, sizeof(int) * 256));
}

static int jacobi_block(int k) { return std::min(kJacobiMaxBS, std::max(1, (k + 15) / 16)); }

bool smallla_fits(const SmallLA& s, int k) { return k <= kSmallLAMaxK && k <= s.kmax; }

namespace {

// 32-row register blocks of the Cholesky and 64-row groups per lane of the
// triangular inverse and Jacobi rounds that k needs (instantiated sizes)
int chol_blocks_for(int k) {
  const int b = (k + kCholT - 1) / kCholT;
  return b <= kCholBSmall ? b : kCholBLarge;
}
int rows_for(int k) {
  const int r = (k + 63) / 64;
  return r <= kRowsSmall ? r : kRowsLarge;
}

void launch_chol(hipStream_t st, int kb, int batch, const double* G, int k, int pass, int shifted, int check_id,
                 double shift_scale, double drop_rel, double* R, double* mask, int* flag) {
  const dim3 grid(batch), block(kCholThreads);
  switch (kb) {
#define CHOL_LAUNCH(KB) \
  case KB:              \
    hipLaunchKernelGGL(k_chol<KB>, grid, block, 0, st, G, k, pass, shifted, check_id, shift_scale, drop_rel, R, mask, flag); \
    break;
    CHOL_LAUNCH(1) CHOL_LAUNCH(2) CHOL_LAUNCH(3) CHOL_LAUNCH(4) CHOL_LAUNCH(5) CHOL_LAUNCH(6)
#undef CHOL_LAUNCH
    default:
      hipLaunchKernelGGL(k_chol<kCholBLarge>, grid, block, 0, st, G, k, pass, shifted, check_id, shift_scale,
                         drop_rel, R, mask, flag);
  }
  CTM_HIP(hipGetLastError());
}

void launch_trinv(hipStream_t st, int rows, int batch, const double* R, const double* mask, int k, double* Ri) {
  const dim3 grid((k + 3) / 4, batch), block(256);
  switch (rows) {
    case 1: hipLaunchKernelGGL(k_trinv<1>, grid, block, 0, st, R, mask, k, Ri); break;
    case 2: hipLaunchKernelGGL(k_trinv<2>, grid, block, 0, st, R, mask, k, Ri); break;
    case 3: hipLaunchKernelGGL(k_trinv<3>, grid, block, 0, st, R, mask, k, Ri); break;
    default: hipLaunchKernelGGL(k_trinv<kRowsLarge>, grid, block, 0, st, R, mask, k, Ri);
  }
  CTM_HIP(hipGetLastError());
}

}  // namespace

void cholqr(hipStream_t st, SmallLA& s, double* Y, long ystride, int n, int k, int batch, int passes,
            double* Racc, const GemmWorkspace& ws) {
  CTM_CHECK(k <= kSmallLAMaxK && k <= s.kmax && batch <= s.batch_max && n >= k, -1, "cholqr: size");
  CTM_CHECK((size_t)n * k * batch <= s.tmp_elems, -1, "cholqr: workspace");
  const long kk2 = (long)k * k;
  const double shift_scale = 11.0 * ((double)n * k + (double)k * (k + 1)) * 0x1p-53;
  double* G = s.G.as<double>();
  double* R = s.R.as<double>();
  double* Ri = s.Rinv.as<double>();
  double* tmp = s.tmp.as<double>();
  double* Rtmp = s.Rtmp.as<double>();
  // the passes alternate between Y and the scratch panels (P holds the
  // current basis); an odd pass count ends with one copy back into Y
  // register blocks and rows per lane sized to k (entries past k are zero
  // and add nothing, so every size gives the same arithmetic)
  const int kb = chol_blocks_for(k), rows = rows_for(k);
  double* P = Y;
  double* Q = tmp;
  long pstride = ystride, qstride = (long)n * k;
  for (int pass = 0; pass < passes; ++pass) {
    // the accumulated factor alternates between Racc and Rtmp so that the
    // last pass leaves it in Racc; the first pass writes its R there directly
    double* rdst = ((passes - 1 - pass) % 2 == 0) ? Racc : Rtmp;
    double* rsrc = (rdst == Racc) ? Rtmp : Racc;
    double* rout = (Racc && pass == 0) ? rdst : R;
    // G = P^T P
    gemm(st, GemmType::F64, k, k, n, 1.0, rowmajor(P, n, pstride), colmajor(P, n, pstride), 0.0,
         out_colmajor(G, k, kk2), batch, ws);
    // the shifted pass never drops; later passes drop a direction only when its
    // pivot (squared residual norm) is below 1e-28 of the largest, i.e. its
    // residual is at the rounding level of the basis (1e-14 relative): such a
    // column is numerically dependent.  Directions damped by the shifted pass
    // are far above that and are kept, as Householder QR keeps them; dropping
    // them at a larger threshold (1e-14 in pivot, 1e-7 in norm) made the kept
    // subspace change from move to move and stalled the corner-spectrum
    // convergence of the iteration.  Only the output of two passes is near
    // orthonormal, so the identity check runs from the third pass on.
    launch_chol(st, kb, batch, G, k, pass, pass == 0 ? 1 : 0, pass >= 2 ? 1 : 0, shift_scale,
                pass == 0 ? 0.0 : 1e-28, rout, s.mask.as<double>(), s.flag.as<int>());
    launch_trinv(st, rows, batch, rout, s.mask.as<double>(), k, Ri);
    CTM_HIP(hipGetLastError());
    // Q = P U^-1 into the other buffer (dropped directions come out zero)
    gemm(st, GemmType::F64, n, k, k, 1.0, colmajor(P, n, pstride), colmajor(Ri, k, kk2), 0.0,
         out_colmajor(Q, n, qstride), batch, ws);
    std::swap(P, Q);
    std::swap(pstride, qstride);
    if (Racc && pass > 0)
      gemm(st, GemmType::F64, k, k, k, 1.0, colmajor(R, k, kk2), colmajor(rsrc, k, kk2), 0.0,
           out_colmajor(rdst, k, kk2), batch, ws);
  }
  if (P != Y) {
    hipLaunchKernelGGL(k_copy_panels, dim3(256, batch), dim3(256), 0, st, P, pstride, Y, ystride, n, k, nullptr);
    CTM_HIP(hipGetLastError());
  }
}

namespace {

// Blocking of the Jacobi for order k: bs columns per block, nb blocks (even).
void jacobi_blocks(int k, int& bs, int& nb) {
  bs = jacobi_block(k);
  nb = (k + bs - 1) / bs;
  if (nb & 1) ++nb;
  if (nb < 2) nb = 2;
}

// At most 14 sweeps; most problems reach the stop in 8, a few in 9, so the
// convergence flags are read back after 8 sweeps and then after each
// further one (rounds of a converged problem return at once, so the
// schedule does not change the results).  Stop: the largest rotated
// |ga| / sqrt(al be) of a sweep at most 1e-10 (the next sweep's would be of
// order 1e-20).
constexpr int kJacobiMaxSweepsVec = 14, kJacobiFirstRead = 8;
constexpr double kJacobiTol = 1e-15, kJacobiStopVec = 1e-10;

void jacobi_vec_sweeps(hipStream_t st, SmallLA& s, double* A, int k, int batch, int count) {
  int bs, nb;
  jacobi_blocks(k, bs, nb);
  double* J = s.J.as<double>();
  int* conv = s.flag.as<int>() + 64;
  int* nsweep = s.flag.as<int>() + 192;
  double* off = s.off.as<double>();
  for (int sw = 0; sw < count; ++sw) {
    for (int r = 0; r < nb - 1; ++r) {
      const dim3 grid(nb / 2, batch), block(64 * bs);
      switch (rows_for(k)) {
        case 1:
        case 2:
          hipLaunchKernelGGL(k_jacobi_round<2>, grid, block, 0, st, A, J, k, nb, bs, r, off, conv, kJacobiTol);
          break;
        case 3:
          hipLaunchKernelGGL(k_jacobi_round<3>, grid, block, 0, st, A, J, k, nb, bs, r, off, conv, kJacobiTol);
          break;
        default:
          hipLaunchKernelGGL(k_jacobi_round<kRowsLarge>, grid, block, 0, st, A, J, k, nb, bs, r, off, conv,
                             kJacobiTol);
      }
    }
    hipLaunchKernelGGL(k_jacobi_sweep_end, dim3(1), dim3(64), 0, st, off, conv, nsweep, batch, kJacobiStopVec);
  }
  CTM_HIP(hipGetLastError());
}

}  // namespace

void jacobi_svd_start(hipStream_t st, SmallLA& s, double* A, int k, int batch) {
  CTM_CHECK(k <= kSmallLAMaxK && batch <= s.batch_max, -1, "jacobi_svd: size");
  double* J = s.J.as<double>();
  if (k <= kJacobiOneWgMaxK) {
    // every sweep of a problem in one workgroup: one launch, no host reads
    hipLaunchKernelGGL((k_jacobi_onewg<64, true>), dim3(batch), dim3(1024), 0, st, A, k, nullptr, J, kJacobiTol,
                       kJacobiStopVec, 14,
                       s.flag.as<int>());
    CTM_HIP(hipGetLastError());
    return;
  }
  int* conv = s.flag.as<int>() + 64;
  int* nsweep = s.flag.as<int>() + 192;
  hipLaunchKernelGGL(k_jacobi_init, dim3(64, batch), dim3(256), 0, st, J, k, s.off.as<double>(), conv, nsweep);
  jacobi_vec_sweeps(st, s, A, k, batch, kJacobiFirstRead);
}

void jacobi_svd_finish(hipStream_t st, SmallLA& s, double* A, int k, int batch, double* X, double* S, long sstride,
                       double* Y) {
  double* J = s.J.as<double>();
  if (k > kJacobiOneWgMaxK) {
    int* conv = s.flag.as<int>() + 64;
    int* nsweep = s.flag.as<int>() + 192;
    for (int done = kJacobiFirstRead; done < kJacobiMaxSweepsVec; ++done) {
      int* hconv = s.hflag.as<int>();
      CTM_HIP(hipMemcpyAsync(hconv, conv, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
      CTM_HIP(hipStreamSynchronize(st));
      bool all = true;
      for (int b = 0; b < batch; ++b) all = all && hconv[b] != 0;
      if (all) break;
      jacobi_vec_sweeps(st, s, A, k, batch, 1);
    }
    hipLaunchKernelGGL(k_jacobi_mark_unconverged, dim3(1), dim3(64), 0, st, conv, s.flag.as<int>(), batch);
    static const bool debug = getenv("CTM_DEBUG") != nullptr;
    if (debug) {
      int* hs = s.hflag.as<int>();
      CTM_HIP(hipMemcpyAsync(hs, nsweep, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
      CTM_HIP(hipMemcpyAsync(hs + 64, conv, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
      CTM_HIP(hipStreamSynchronize(st));
      const int* h[2] = {hs, hs + 64};
      fprintf(stderr, "[ctm] jacobi k=%d:", k);
      for (int b = 0; b < batch; ++b) fprintf(stderr, " %d%s", h[0][b], h[1][b] ? "" : "(not converged)");
      fprintf(stderr, "\n");
    }
  }
  hipLaunchKernelGGL(k_svd_finalize, dim3(batch), dim3(256), 0, st, A, J, k, X, S, sstride, Y);
  CTM_HIP(hipGetLastError());
}

void jacobi_svd(hipStream_t st, SmallLA& s, double* A, int k, int batch, double* X, double* S, long sstride,
                double* Y) {
  jacobi_svd_start(st, s, A, k, batch);
  jacobi_svd_finish(st, s, A, k, batch, X, S, sstride, Y);
}


void singular_values_batched(hipStream_t st, double* A, int k, int batch, double* S, long sstride, double* off,
                             int* conv, int* nsweep, int* hconv) {
  CTM_CHECK(k >= 1 && k <= kSmallLAMaxK && batch >= 1 && batch <= 64, -1, "singular_values_batched: size");
  int bs = jacobi_block(k);
  int nb = (k + bs - 1) / bs;
  if (nb & 1) ++nb;
  if (nb < 2) nb = 2;
  const double tol = 1e-15;
  hipLaunchKernelGGL(k_jacobi_init_values, dim3(1), dim3(64), 0, st, off, conv, nsweep, batch);
  // values only: their error is of order the square of the remaining
  // |ga| / sqrt(al be), so a sweep whose rotations stayed below 1e-8 ends it
  const int max_sweeps = 30, first = 7;
  const double stop = 1e-8;
  auto sweeps = [&](int count) {
    for (int sw = 0; sw < count; ++sw) {
      for (int r = 0; r < nb - 1; ++r) {
        const dim3 grid(nb / 2, batch), block(64 * bs);
        switch (rows_for(k)) {
          case 1:
          case 2:
            hipLaunchKernelGGL((k_jacobi_round<2, false>), grid, block, 0, st, A, nullptr, k, nb, bs, r, off, conv, tol);
            break;
          case 3:
            hipLaunchKernelGGL((k_jacobi_round<3, false>), grid, block, 0, st, A, nullptr, k, nb, bs, r, off, conv, tol);
            break;
          default:
            hipLaunchKernelGGL((k_jacobi_round<kRowsLarge, false>), grid, block, 0, st, A, nullptr, k, nb, bs, r, off,
                               conv, tol);
        }
      }
      hipLaunchKernelGGL(k_jacobi_sweep_end, dim3(1), dim3(64), 0, st, off, conv, nsweep, batch, stop);
    }
    CTM_HIP(hipGetLastError());
  };
  // rounds of a converged problem return at once: reading the flags after
  // `first` sweeps and then after each further one does not change results
  sweeps(first);
  for (int done = first; done < max_sweeps; ++done) {
    CTM_HIP(hipMemcpyAsync(hconv, conv, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
    CTM_HIP(hipStreamSynchronize(st));
    bool all = true;
    for (int b = 0; b < batch; ++b) all = all && hconv[b] != 0;
    if (all) break;
    sweeps(1);
  }
  hipLaunchKernelGGL(k_colnorm_desc, dim3(batch), dim3(256), 0, st, A, k, S, sstride);
  CTM_HIP(hipGetLastError());
}

void singular_values_small(hipStream_t st, const double* A, int m, int batch, double* S) {
  CTM_CHECK(m >= 1 && m <= kSvSmallMax && batch >= 1, -1, "singular_values_small: size");
  // the kernel reads A and writes only S; rows per lane sized to m
  if (m <= 64)
    hipLaunchKernelGGL((k_jacobi_onewg<64, false>), dim3(batch), dim3(1024), 0, st, const_cast<double*>(A), m, S,
                       nullptr, 1e-15, 0.0, 30, nullptr);
  else
    hipLaunchKernelGGL((k_jacobi_onewg<kSvSmallMax, false>), dim3(batch), dim3(1024), 0, st, const_cast<double*>(A), m,
                       S, nullptr, 1e-15, 0.0, 30, nullptr);
  CTM_HIP(hipGetLastError());
}

}  // namespace ctm
