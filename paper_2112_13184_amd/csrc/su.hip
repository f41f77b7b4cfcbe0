// Simple-update imaginary-time evolution and the mean-field environment
// (Sec. 2.3, Eqs. (1)-(4); Sec. 2.2, mean-field environment).
//
// A batch of independent problems (for instance one per field value of a
// phase scan) evolves at once: one workgroup per problem runs every Trotter
// step and every bond of its unit cell in order, with the reduced tensors of
// the bond in LDS.  Bond update (i, j, weight lam on the shared bond k):
//   M_i[a][(k, p)] = G_i with the weights of its three other legs a absorbed
//                    (rows D^3, columns D d), likewise M_j;
//   M_i = Q_i R_i, M_j = Q_j R_j          Householder QR in LDS;
//   Theta[(x, P)][(y, Q)] = sum_{p q} g[(P Q)][(p q)] sum_k R_i[x][(k p)] lam[k] R_j[y][(k q)];
//   Theta = U S V^T                       one-sided Jacobi in LDS;
//   keep the D largest, lam' = S / ||S||_2,
//   G_i' = (Q_i U)[(a, P)][k] / weights(a), G_j' = (Q_j V) likewise.
// The product Q_i U is the left factor of the SVD of the full two-site
// matrix (D^3 d rows), so the sign of each kept pair is fixed on it: the first
// entry in (a, P) order whose modulus is within 1e-8 of the largest is made
// positive.  A weight <= 1e-13 is divided out as zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "ctm.h"
#include "wave.hpp"

namespace ctm {
namespace {

constexpr int kSuThreads = 256;
constexpr int kSuWaves = kSuThreads / 64;
constexpr double kSuInvCut = 1e-13;
constexpr double kSuSignTol = 1e-8;
constexpr double kSuJacobiTol = 1e-15;
constexpr double kSuJacobiStop = 1e-10;
constexpr double kSuJacobiZero = 1e-30;
constexpr int kSuJacobiMaxSweeps = 40;
constexpr int kSuStepsPerLaunch = 64;

struct SuShape {
  int Lx, Ly, N, D, d, d2, R, C, k, m, np;
};

__host__ __device__ inline SuShape su_shape(int Lx, int Ly, int D, int d) {
  SuShape s;
  s.Lx = Lx; s.Ly = Ly; s.N = Lx * Ly; s.D = D; s.d = d; s.d2 = d * d;
  s.R = D * D * D;
  s.C = D * d;
  s.k = s.R < s.C ? s.R : s.C;
  s.m = s.k * d;
  s.np = s.m + (s.m & 1);
  return s;
}


struct SuArgs {
  double* gamma;        // [batch][N][D^4 d]
  double* lam;          // [batch][N][2][D]
  const double* gates;  // [batch][N][2][d^2][d^2]
  int* status;          // [batch]: bit 0 = a bond had no singular value above zero or a non-finite one
  int Lx, Ly, D, d, nsteps;
};

// legs of a site other than `leg`, in leg order
__device__ inline int other_leg(int leg, int t) {
  return t == 0 ? (leg == 0 ? 1 : 0) : t == 1 ? (leg <= 1 ? 2 : 1) : (leg <= 2 ? 3 : 2);
}
// element stride of leg l (0..3) in G[l][u][r][d][p]
__device__ inline long leg_stride(int leg, int D, int d) {
  return leg == 0 ? (long)D * D * D * d : leg == 1 ? (long)D * D * d : leg == 2 ? (long)D * d : (long)d;
}
// weights on leg `lg` of `site` (l: right bond of the left neighbour, u: own
// upper bond, r: own right bond, d: upper bond of the lower neighbour)
__device__ inline const double* leg_weight(const double* lamL, int site, int lg, int Lx, int Ly, int D) {
  const int sx = site % Lx, sy = site / Lx;
  switch (lg) {
    case 0: return lamL + (((sx - 1 + Lx) % Lx + Lx * sy) * 2 + 0) * D;
    case 1: return lamL + (site * 2 + 1) * D;
    case 2: return lamL + (site * 2 + 0) * D;
    default: return lamL + ((sx + Lx * ((sy - 1 + Ly) % Ly)) * 2 + 1) * D;
  }
}

// 1 / sqrt(x), x > 0 normal: the hardware estimate and two Newton steps
// y += y (1 - x y^2) / 2 (each roughly doubles the correct bits).
__device__ inline double su_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double h = x * y;
    const double e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Sum over aligned groups of TL lanes (TL = 1, 2, 4, 8 or 16) inside the
// 16-lane DPP rows; every lane of a group receives its group's sum.  All 64
// lanes must be active.
__device__ inline double group_sum(double v, int TL) {
  if (TL >= 2) v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  if (TL >= 4) v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  if (TL >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
  if (TL >= 16) v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

__device__ inline int imin_wave(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off));
  return v;
}

// Scalars of the tensors: FP64 real, or FP64 complex (re, im interleaved in
// memory).  The helpers reduce to plain real arithmetic for double.
struct zc {
  double re, im;
};
__host__ __device__ inline zc operator+(zc a, zc b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline zc operator-(zc a, zc b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline zc operator*(zc a, zc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline zc operator*(double s, zc a) { return {s * a.re, s * a.im}; }
__host__ __device__ inline zc operator*(zc a, double s) { return {s * a.re, s * a.im}; }
__host__ __device__ inline zc& operator+=(zc& a, zc b) { a.re += b.re; a.im += b.im; return a; }
__host__ __device__ inline zc& operator-=(zc& a, zc b) { a.re -= b.re; a.im -= b.im; return a; }
__host__ __device__ inline zc& operator*=(zc& a, zc b) { a = a * b; return a; }
__host__ __device__ inline zc& operator*=(zc& a, double s) { a.re *= s; a.im *= s; return a; }

template <typename T> __device__ inline T szero();
template <> __device__ inline double szero<double>() { return 0.0; }
template <> __device__ inline zc szero<zc>() { return {0.0, 0.0}; }
template <typename T> __device__ inline T sreal(double x);
template <> __device__ inline double sreal<double>(double x) { return x; }
template <> __device__ inline zc sreal<zc>(double x) { return {x, 0.0}; }
__device__ inline double sre(double a) { return a; }
__device__ inline double sre(zc a) { return a.re; }
__device__ inline double sabs2(double a) { return a * a; }
__device__ inline double sabs2(zc a) { return a.re * a.re + a.im * a.im; }
__device__ inline double sabs(double a) { return fabs(a); }
__device__ inline double sabs(zc a) { return sqrt(sabs2(a)); }
__device__ inline double sconj(double a) { return a; }
__device__ inline zc sconj(zc a) { return {a.re, -a.im}; }
__device__ inline bool siszero(double a) { return a == 0.0; }
__device__ inline bool siszero(zc a) { return a.re == 0.0 && a.im == 0.0; }
// conj(a) b
__device__ inline double cmul(double a, double b) { return a * b; }
__device__ inline zc cmul(zc a, zc b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }
__device__ inline double srecip(double a) { return 1.0 / a; }
__device__ inline zc srecip(zc a) {
  const double n = 1.0 / sabs2(a);
  return {a.re * n, -a.im * n};
}
__device__ inline double wave_sum_s(double v) { return wave_sum(v); }
__device__ inline zc wave_sum_s(zc v) { return {wave_sum(v.re), wave_sum(v.im)}; }
__device__ inline double group_sum_s(double v, int TL) { return group_sum(v, TL); }
__device__ inline zc group_sum_s(zc v, int TL) { return {group_sum(v.re, TL), group_sum(v.im, TL)}; }

// doubles of LDS one bond update needs (scalar arrays count sizeof(T) / 8 each)
__host__ __device__ inline long su_lds_need(const SuShape& s, int words) {
  return words * (2L * s.R * s.C + (long)s.m * s.np + (long)s.np * s.np + 3L * s.C + s.D) + 2L * s.N * s.D + s.np +
         s.C + s.D + 8;
}

// CAP doubles of LDS; each wave keeps CPW columns of RPL rows per lane of the
// reconstructed tensors in registers (D^3 <= 64 RPL, D d <= 4 CPW).
template <typename T, int CAP, int RPL, int CPW>
__global__ __launch_bounds__(kSuThreads) void k_su_run(SuArgs a) {
  constexpr int kSuMaxRowsPerLane = RPL;
  constexpr int kSuMaxColsPerWave = CPW;
  constexpr bool kReal = sizeof(T) == sizeof(double);
  __shared__ __attribute__((aligned(16))) double lds[CAP];
  __shared__ int ip[64 + 32 + 2];
  const SuShape S = su_shape(a.Lx, a.Ly, a.D, a.d);
  const int D = S.D, d = S.d, R = S.R, C = S.C, k = S.k, m = S.m, np = S.np, N = S.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.x;
  const long T_ = (long)R * D * d;
  T* G = reinterpret_cast<T*>(a.gamma) + (long)b * N * T_;
  double* lamG = a.lam + (long)b * N * 2 * D;
  const T* gates = reinterpret_cast<const T*>(a.gates) + (long)b * N * 2 * S.d2 * S.d2;

  T* Mi = reinterpret_cast<T*>(lds);
  T* Mj = Mi + (long)R * C;
  T* Th = Mj + (long)R * C;            // m x np, column-major
  T* Vv = Th + (long)m * np;           // np x np, column-major
  T* taui = Vv + (long)np * np;        // C
  T* tauj = taui + C;                  // C
  T* cval = tauj + C;                  // C
  T* flip = cval + C;                  // D: phase of each kept pair
  double* lamL = reinterpret_cast<double*>(flip + D);   // [N][2][D]
  double* sig = lamL + 2 * N * D;      // np
  double* cmax = sig + np;             // C
  double* lamN = cmax + C;             // D
  int* perm = ip;                      // D (<= 64 entries reserved)
  int* cand = ip + 64;                 // C (<= 32)

  for (int e = tid; e < 2 * N * D; e += kSuThreads) lamL[e] = lamG[e];
  int bad = 0;
  __syncthreads();

  for (int step = 0; step < a.nsteps; ++step) {
    for (int dir = 0; dir < 2; ++dir) {
      for (int s = 0; s < N; ++s) {
        const int x = s % S.Lx, y = s / S.Lx;
        const int si = s, li = dir == 0 ? 2 : 1;
        const int sj = dir == 0 ? (x + 1) % S.Lx + S.Lx * y : x + S.Lx * ((y + 1) % S.Ly);
        const int lj = dir == 0 ? 0 : 3;
        const double* lamB = lamL + (s * 2 + dir) * D;
        const T* g = gates + (long)(s * 2 + dir) * S.d2 * S.d2;
        // weights and strides of the three other legs of i and j, in leg order
        const double* wi0 = leg_weight(lamL, si, other_leg(li, 0), S.Lx, S.Ly, D);
        const double* wi1 = leg_weight(lamL, si, other_leg(li, 1), S.Lx, S.Ly, D);
        const double* wi2 = leg_weight(lamL, si, other_leg(li, 2), S.Lx, S.Ly, D);
        const double* wj0 = leg_weight(lamL, sj, other_leg(lj, 0), S.Lx, S.Ly, D);
        const double* wj1 = leg_weight(lamL, sj, other_leg(lj, 1), S.Lx, S.Ly, D);
        const double* wj2 = leg_weight(lamL, sj, other_leg(lj, 2), S.Lx, S.Ly, D);
        const long si0 = leg_stride(other_leg(li, 0), D, d), si1 = leg_stride(other_leg(li, 1), D, d);
        const long si2 = leg_stride(other_leg(li, 2), D, d), sib = leg_stride(li, D, d);
        const long sj0 = leg_stride(other_leg(lj, 0), D, d), sj1 = leg_stride(other_leg(lj, 1), D, d);
        const long sj2 = leg_stride(other_leg(lj, 2), D, d), sjb = leg_stride(lj, D, d);
        T* Gi = G + (long)si * T_;
        T* Gj = G + (long)sj * T_;

        // ---- M_i, M_j (column-major, column c = k d + p) ----
        for (long e = tid; e < (long)R * C; e += kSuThreads) {
          const int r = (int)(e % R), c = (int)(e / R);
          const int a1 = r / (D * D), a2 = (r / D) % D, a3 = r % D;
          const int kk = c / d, p = c % d;
          Mi[e] = Gi[a1 * si0 + a2 * si1 + a3 * si2 + kk * sib + p] * (wi0[a1] * wi1[a2] * wi2[a3]);
          Mj[e] = Gj[a1 * sj0 + a2 * sj1 + a3 * sj2 + kk * sjb + p] * (wj0[a1] * wj1[a2] * wj2[a3]);
        }
        __syncthreads();

        // ---- Householder QR of M_i and M_j (2 C columns over the waves) ----
        // The wave that owns column c applies reflector j to it in step j and,
        // if c = j + 1, then forms reflector j + 1 from it: one barrier a step.
        // H_j = I - tau_j v_j v_j^H with v_j[j] = 1 and H_j^H x = beta e_j,
        // beta real; the factorisation applies H_j^H, so M = Q R with
        // Q = H_0 H_1 ...
        auto make_reflector = [&](T* M, T* tau, int j) {
          T* col = M + (long)j * R;
          double part = 0.0;
#pragma unroll
          for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
            const int r = lane + 64 * t;
            if (r > j && r < R) part += sabs2(col[r]);
          }
          const double xn2 = wave_sum(part);
          const T alpha = col[j];
          if (xn2 == 0.0) {
            if (lane == 0) tau[j] = szero<T>();
            return;
          }
          const double beta = -copysign(sqrt(sabs2(alpha) + xn2), sre(alpha));
          const T sc = srecip(alpha - sreal<T>(beta));
#pragma unroll
          for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
            const int r = lane + 64 * t;
            if (r > j && r < R) col[r] *= sc;
          }
          if (lane == 0) { tau[j] = (sreal<T>(beta) - alpha) * (1.0 / beta); col[j] = sreal<T>(beta); }
        };
        auto apply_reflector = [&](T* M, const T* tau, int j, int c) {
          const T tj = tau[j];
          if (siszero(tj)) return;
          const T* v = M + (long)j * R;
          T* col = M + (long)c * R;
          T part = szero<T>();
#pragma unroll
          for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
            const int r = lane + 64 * t;
            if (r >= j && r < R) part += (r == j ? col[r] : cmul(v[r], col[r]));
          }
          const T w = sconj(tj) * wave_sum_s(part);
#pragma unroll
          for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
            const int r = lane + 64 * t;
            if (r >= j && r < R) col[r] -= (r == j ? w : w * v[r]);
          }
        };
        if (wave == 0) make_reflector(Mi, taui, 0);
        if (wave == (C % kSuWaves)) make_reflector(Mj, tauj, 0);
        __syncthreads();
        for (int j = 0; j < k; ++j) {
          for (int gcol = wave; gcol < 2 * C; gcol += kSuWaves) {
            const bool left = gcol < C;
            const int c = left ? gcol : gcol - C;
            if (c <= j) continue;
            T* M = left ? Mi : Mj;
            T* tau = left ? taui : tauj;
            apply_reflector(M, tau, j, c);
            if (c == j + 1 && j + 1 < k) make_reflector(M, tau, j + 1);
          }
          __syncthreads();
        }

        // ---- Theta = gate applied to R_i lam R_j^T; V = identity ----
        for (int e = tid; e < m * np; e += kSuThreads) {
          const int r = e % m, cI = e / m;
          T val = szero<T>();
          if (cI < m) {
            const int xr = r / d, P = r % d, yc = cI / d, Q = cI % d;
            for (int p = 0; p < d; ++p) {
              for (int q = 0; q < d; ++q) {
                const T gv = g[(P * d + Q) * S.d2 + p * d + q];
                if (siszero(gv)) continue;
                T t = szero<T>();
                for (int kk = 0; kk < D; ++kk) {
                  const int ca = kk * d + p, cb = kk * d + q;
                  const T ri = xr <= ca ? Mi[(long)ca * R + xr] : szero<T>();
                  const T rj = yc <= cb ? Mj[(long)cb * R + yc] : szero<T>();
                  t += ri * lamB[kk] * rj;
                }
                val += gv * t;
              }
            }
          }
          Th[e] = val;
        }
        for (int e = tid; e < np * np; e += kSuThreads) Vv[e] = sreal<T>((e % np) == (e / np) ? 1.0 : 0.0);
        __syncthreads();

        // ---- one-sided Jacobi on the columns of Theta (round-robin pairs) ----
        // One wave runs every round: the np / 2 pairs of a round go to groups
        // of TL lanes (the largest power of two <= 16 with np / 2 groups in 64
        // lanes) inside the 16-lane DPP rows, whose sums take log2(TL) DPP
        // steps; the wave's LDS accesses stay in program order, so the rounds
        // need no barrier.
        if (wave == 0) {
          const int P = np / 2;
          int TL = 16;                        // a power of two: groups stay inside DPP rows
          while (TL * P > 64) TL >>= 1;
          const int grp = lane / TL, gl = lane % TL;
          const bool active = grp < P;
          // columns with |c|^2 <= 1e-30 ||Theta||_F^2 are rounding noise: no rotation
          double fro = 0.0;
          for (int e = lane; e < m * m; e += 64) fro += sabs2(Th[e]);
          const double tiny = kSuJacobiZero * wave_sum(fro);
          for (int sw = 0; sw < kSuJacobiMaxSweeps; ++sw) {
            int rotated = 0, large = 0;         // any rotation; any with |gamma| > 1e-10 sqrt(alpha beta)
            for (int rd = 0; rd < np - 1; ++rd) {
              // round-robin pairs; for the active groups rd + grp and
              // rd - grp + np - 1 lie in [0, 2 (np - 1)), so one conditional
              // subtraction reduces them (inactive lanes keep column 0)
              int pa = 0, pb = 0;
              if (grp == 0) { pa = np - 1; pb = rd; }
              else if (active) {
                pa = rd + grp;
                pa = pa >= np - 1 ? pa - (np - 1) : pa;
                pb = rd - grp + np - 1;
                pb = pb >= np - 1 ? pb - (np - 1) : pb;
              }
              T* ca = Th + (long)pa * m;
              T* cb = Th + (long)pb * m;
              double al = 0.0, be = 0.0;
              T ga = szero<T>();
              if (active) {
                for (int r = gl; r < m; r += TL) {
                  const T u = ca[r], v = cb[r];
                  al += sabs2(u); be += sabs2(v); ga += cmul(u, v);
                }
              }
              al = group_sum(al, TL);
              be = group_sum(be, TL);
              ga = group_sum_s(ga, TL);
              const double g2 = sabs2(ga), ab = al * be;
              if (active && g2 != 0.0 && al > tiny && be > tiny && g2 > kSuJacobiTol * kSuJacobiTol * ab) {
                large |= g2 > kSuJacobiStop * kSuJacobiStop * ab;
                // the angle zeroing the inner product: tan(2 theta) = 2 |ga| / (be - al);
                // with dd = be - al, q = sqrt(dd^2 + 4 |ga|^2), w = sqrt(2 q (q + |dd|)):
                // cos = (q + |dd|) / w, sin = 2 |ga| sgn(dd) / w, from two reciprocal
                // square roots and no division
                const double dd = be - al, ad = fabs(dd);
                const double X = dd * dd + 4.0 * g2;
                const double q = X * su_rsqrt(X);
                const double inv = su_rsqrt(2.0 * q * (q + ad));
                const double cs = (q + ad) * inv;
                double* va0 = nullptr;
                (void)va0;
                T* va = Vv + (long)pa * np;
                T* vb = Vv + (long)pb * np;
                if constexpr (kReal) {
                  const double sn = 2.0 * sre(ga) * (dd >= 0.0 ? inv : -inv);
                  for (int r = gl; r < m; r += TL) {
                    const double u = sre(ca[r]), v = sre(cb[r]);
                    ca[r] = sreal<T>(cs * u - sn * v);
                    cb[r] = sreal<T>(sn * u + cs * v);
                  }
                  for (int r = gl; r < np; r += TL) {
                    const double u = sre(va[r]), v = sre(vb[r]);
                    va[r] = sreal<T>(cs * u - sn * v);
                    vb[r] = sreal<T>(sn * u + cs * v);
                  }
                } else {
                  // the real rotation of (a, ph b), ph = conj(ga) / |ga|, whose inner
                  // product is |ga|: a' = cs a - sigma b, b' = sn a + cs ph b
                  const double gabs = sqrt(g2);
                  const T ph = sconj(ga) * (1.0 / gabs);
                  const double sn = 2.0 * gabs * (dd >= 0.0 ? inv : -inv);
                  const T sigma = ph * sn;
                  for (int r = gl; r < m; r += TL) {
                    const T u = ca[r], v = cb[r];
                    ca[r] = u * cs - sigma * v;
                    cb[r] = u * sn + (ph * v) * cs;
                  }
                  for (int r = gl; r < np; r += TL) {
                    const T u = va[r], v = vb[r];
                    va[r] = u * cs - sigma * v;
                    vb[r] = u * sn + (ph * v) * cs;
                  }
                }
                rotated = 1;
              }
              __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
            // quadratic convergence: after a sweep whose rotations were all
            // below 1e-10 the remaining off-diagonal terms are ~1e-20
            if (!__any(rotated) || !__any(large)) break;
          }
        }
        __syncthreads();

        // ---- singular values, the D largest, new weights ----
        for (int c = tid; c < m; c += kSuThreads) {
          double ss = 0.0;
          for (int r = 0; r < m; ++r) ss += sabs2(Th[(long)c * m + r]);
          sig[c] = sqrt(ss);
        }
        __syncthreads();
        for (int c = tid; c < m; c += kSuThreads) {
          const double sc = sig[c];
          int rank = 0;
          for (int c2 = 0; c2 < m; ++c2) {
            const double s2 = sig[c2];
            rank += (s2 > sc) || (s2 == sc && c2 < c);
          }
          if (rank < D) perm[rank] = c;
        }
        __syncthreads();
        double nrm = 0.0;
        for (int kk = 0; kk < D; ++kk) nrm += sig[perm[kk]] * sig[perm[kk]];
        nrm = sqrt(nrm);
        if (!(nrm > 0.0) || !isfinite(nrm)) bad = 1;
        if (tid < D) lamN[tid] = nrm > 0.0 ? sig[perm[tid]] / nrm : 0.0;

        // ---- G_i' = Q_i U (columns (k', P) in registers), phase rule ----
        T yv[kSuMaxColsPerWave][kSuMaxRowsPerLane];
        auto apply_q = [&](const T* M, const T* tau, T (&yy)[kSuMaxRowsPerLane]) {
          for (int j = k - 1; j >= 0; --j) {
            const T tj = tau[j];
            if (siszero(tj)) continue;
            const T* v = M + (long)j * R;
            T part = szero<T>();
#pragma unroll
            for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
              const int r = lane + 64 * t;
              if (r >= j && r < R) part += (r == j ? yy[t] : cmul(v[r], yy[t]));
            }
            const T w = tj * wave_sum_s(part);
#pragma unroll
            for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
              const int r = lane + 64 * t;
              if (r >= j && r < R) yy[t] -= (r == j ? w : w * v[r]);
            }
          }
        };
#pragma unroll
        for (int q = 0; q < kSuMaxColsPerWave; ++q) {
          const int cc = wave + kSuWaves * q;
          if (cc < C) {
            const int kk = cc / d, P = cc % d;
            const int pc = perm[kk];
            const double sv = sig[pc];
            const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
#pragma unroll
            for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
              const int r = lane + 64 * t;
              yv[q][t] = r < k ? Th[(long)pc * m + r * d + P] * inv : szero<T>();
            }
            apply_q(Mi, taui, yv[q]);
            double mx = 0.0;
#pragma unroll
            for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
              const int r = lane + 64 * t;
              if (r < R) mx = fmax(mx, sabs(yv[q][t]));
            }
            mx = wave_max(mx);
            if (lane == 0) cmax[cc] = mx;
          }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kSuMaxColsPerWave; ++q) {
          const int cc = wave + kSuWaves * q;
          if (cc < C) {
            const int kk = cc / d, P = cc % d;
            double gmax = 0.0;
            for (int p2 = 0; p2 < d; ++p2) gmax = fmax(gmax, cmax[kk * d + p2]);
            const double thr = (1.0 - kSuSignTol) * gmax;
            int best = 1 << 30;
#pragma unroll
            for (int t = kSuMaxRowsPerLane - 1; t >= 0; --t) {
              const int r = lane + 64 * t;
              if (r < R && sabs(yv[q][t]) >= thr) best = r;
            }
            best = imin_wave(best);
#pragma unroll
            for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
              const int r = lane + 64 * t;
              if (r == best) cval[cc] = yv[q][t];
            }
            if (lane == 0) cand[cc] = best < (1 << 30) ? best * d + P : (1 << 30);
          }
        }
        __syncthreads();
        if (tid < D) {
          // the phase that makes the chosen entry real and positive (a sign for
          // real tensors)
          int bi = 1 << 30;
          T bv = szero<T>();
          for (int p2 = 0; p2 < d; ++p2) {
            const int c2 = tid * d + p2;
            if (cand[c2] < bi) { bi = cand[c2]; bv = cval[c2]; }
          }
          if constexpr (kReal) {
            flip[tid] = sreal<T>(sre(bv) < 0.0 ? -1.0 : 1.0);
          } else {
            const double ab = sabs(bv);
            flip[tid] = ab > 0.0 ? sconj(bv) * (1.0 / ab) : sreal<T>(1.0);
          }
        }
        __syncthreads();
        // write G_i'
#pragma unroll
        for (int q = 0; q < kSuMaxColsPerWave; ++q) {
          const int cc = wave + kSuWaves * q;
          if (cc < C) {
            const int kk = cc / d, P = cc % d;
            const T f = flip[kk];
#pragma unroll
            for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
              const int r = lane + 64 * t;
              if (r < R) {
                const int a1 = r / (D * D), a2 = (r / D) % D, a3 = r % D;
                const double w0 = wi0[a1], w1 = wi1[a2], w2 = wi2[a3];
                const double iw = (w0 > kSuInvCut && w1 > kSuInvCut && w2 > kSuInvCut) ? 1.0 / (w0 * w1 * w2) : 0.0;
                Gi[a1 * si0 + a2 * si1 + a3 * si2 + kk * sib + P] = (f * yv[q][t]) * iw;
              }
            }
          }
        }
        // G_j' = Q_j conj(V) with the conjugate phases
#pragma unroll
        for (int q = 0; q < kSuMaxColsPerWave; ++q) {
          const int cc = wave + kSuWaves * q;
          if (cc < C) {
            const int kk = cc / d, Qp = cc % d;
            const int pc = perm[kk];
#pragma unroll
            for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
              const int r = lane + 64 * t;
              yv[q][t] = r < k ? sconj(Vv[(long)pc * np + r * d + Qp]) : szero<T>();
            }
            apply_q(Mj, tauj, yv[q]);
            const T f = sconj(flip[kk]);
#pragma unroll
            for (int t = 0; t < kSuMaxRowsPerLane; ++t) {
              const int r = lane + 64 * t;
              if (r < R) {
                const int a1 = r / (D * D), a2 = (r / D) % D, a3 = r % D;
                const double w0 = wj0[a1], w1 = wj1[a2], w2 = wj2[a3];
                const double iw = (w0 > kSuInvCut && w1 > kSuInvCut && w2 > kSuInvCut) ? 1.0 / (w0 * w1 * w2) : 0.0;
                Gj[a1 * sj0 + a2 * sj1 + a3 * sj2 + kk * sjb + Qp] = (f * yv[q][t]) * iw;
              }
            }
          }
        }
        __syncthreads();
        if (tid < D) lamL[(s * 2 + dir) * D + tid] = lamN[tid];
        __syncthreads();
      }
    }
  }
  for (int e = tid; e < 2 * N * D; e += kSuThreads) lamG[e] = lamL[e];
  if (bad) atomicOr(a.status + b, 1);
}

// exp(-tau H) of every bond Hamiltonian: one workgroup per gate, scaling and
// squaring of a degree-18 Taylor polynomial (Horner form) at norm <= 1/4.
template <typename T>
__global__ __launch_bounds__(256) void k_su_gates(const double* Hd, const double* tau, double* gatesd, int N, int d2) {
  __shared__ T X[256], Pm[256], W[256];
  __shared__ int sq;
  const T* H = reinterpret_cast<const T*>(Hd);
  T* gates = reinterpret_cast<T*>(gatesd);
  const int gidx = blockIdx.x;                 // (b * N + s) * 2 + dir
  const int b = gidx / (2 * N);
  const int n = d2, nn = d2 * d2, tid = threadIdx.x;
  const T* h = H + (long)gidx * nn;
  const double t = tau[b];
  if (tid < nn) X[tid] = h[tid] * (-t);
  __syncthreads();
  if (tid == 0) {
    double nrm = 0.0;                          // 1-norm (largest column sum)
    for (int c = 0; c < n; ++c) {
      double cs = 0.0;
      for (int r = 0; r < n; ++r) cs += sabs(X[r * n + c]);
      nrm = fmax(nrm, cs);
    }
    int s = 0;
    while (nrm > 0.25 && s < 60) { nrm *= 0.5; ++s; }
    sq = s;
  }
  __syncthreads();
  const double scale = ldexp(1.0, -sq);
  if (tid < nn) { X[tid] = X[tid] * scale; Pm[tid] = sreal<T>((tid / n == tid % n) ? 1.0 : 0.0); }
  __syncthreads();
  for (int kdeg = 18; kdeg >= 1; --kdeg) {
    if (tid < nn) {
      const int r = tid / n, c = tid % n;
      T acc = szero<T>();
      for (int q = 0; q < n; ++q) acc += X[r * n + q] * Pm[q * n + c];
      W[tid] = sreal<T>(r == c ? 1.0 : 0.0) + acc * (1.0 / kdeg);
    }
    __syncthreads();
    if (tid < nn) Pm[tid] = W[tid];
    __syncthreads();
  }
  for (int it = 0; it < sq; ++it) {
    if (tid < nn) {
      const int r = tid / n, c = tid % n;
      T acc = szero<T>();
      for (int q = 0; q < n; ++q) acc += Pm[r * n + q] * Pm[q * n + c];
      W[tid] = acc;
    }
    __syncthreads();
    if (tid < nn) Pm[tid] = W[tid];
    __syncthreads();
  }
  if (tid < nn) gates[(long)gidx * nn + tid] = Pm[tid];
}

// Mean-field environment (Sec. 2.2): blockIdx.y = 0 gives the one-site
// density matrix of site blockIdx.x (weights squared on all four legs),
// 1 / 2 the bond to its right / upper neighbour:
//   K_s[(k p)][(k' p')] = sum_a A_s[a, k, p] conj(A_s[a, k', p']) (A_s = G_s with
//   its three other legs weighted), rho[(p q)][(p' q')] = sum_{k k'} K_i lam_k lam_k' K_j.
// Both are normalised to unit trace; rho[ket][bra].
// scalars of LDS for the weighted tensor A (D^3 x D d) of the bond kind
template <typename T> constexpr int mfe_a_cap() { return sizeof(T) == sizeof(double) ? 8192 : 4096; }
template <typename T>
__global__ __launch_bounds__(256) void k_su_mfe(const double* gammad, const double* lam, double* rho1d, double* rho2d,
                                                int Lx, int Ly, int D, int d) {
  constexpr int kA = mfe_a_cap<T>();
  __shared__ __attribute__((aligned(16))) double shd[(kA + 2 * 1024 + 256 + 64) * (sizeof(T) / sizeof(double))];
  T* sh = reinterpret_cast<T*>(shd);
  const T* gamma = reinterpret_cast<const T*>(gammad);
  T* rho1 = reinterpret_cast<T*>(rho1d);
  T* rho2 = reinterpret_cast<T*>(rho2d);
  const int N = Lx * Ly, s = blockIdx.x, kind = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
  const int R = D * D * D, C = D * d, d2 = d * d;
  const long T_ = (long)R * D * d;
  const T* G = gamma + (long)b * N * T_;
  const double* lamL = lam + (long)b * N * 2 * D;
  auto wptr = [&](int site, int lg) { return leg_weight(lamL, site, lg, Lx, Ly, D); };
  T* red = sh + kA + 2048;     // 256 + 64
  if (kind == 0) {
    const T* Gs = G + (long)s * T_;
    const double* w0 = wptr(s, 0); const double* w1 = wptr(s, 1);
    const double* w2 = wptr(s, 2); const double* w3 = wptr(s, 3);
    // each thread accumulates d^2 partial sums over its leg combinations
    for (int pp = 0; pp < d2; ++pp) {
      const int p = pp / d, p2 = pp % d;
      T acc = szero<T>();
      for (long e = tid; e < (long)R * D; e += 256) {
        const int l = (int)(e / (D * D * D)), u = (int)((e / (D * D)) % D), r = (int)((e / D) % D), dd = (int)(e % D);
        const double w = w0[l] * w1[u] * w2[r] * w3[dd];
        const long base = e * d;
        acc += cmul(Gs[base + p2], Gs[base + p]) * (w * w);
      }
      red[tid] = acc;
      __syncthreads();
      for (int h = 128; h >= 1; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
      }
      if (tid == 0) sh[pp] = red[0];
      __syncthreads();
    }
    if (tid < d2) {
      double tr = 0.0;
      for (int p = 0; p < d; ++p) tr += sre(sh[p * d + p]);
      rho1[((long)b * N + s) * d2 + tid] = sh[tid] * (1.0 / tr);
    }
    return;
  }
  const int dir = kind - 1;
  const int x = s % Lx, y = s / Lx;
  const int si = s, li = dir == 0 ? 2 : 1;
  const int sj = dir == 0 ? (x + 1) % Lx + Lx * y : x + Lx * ((y + 1) % Ly);
  const int lj = dir == 0 ? 0 : 3;
  const double* lamB = lamL + (s * 2 + dir) * D;
  T* A = sh;                            // R x C
  T* Ki = sh + kA;                      // C x C
  T* Kj = Ki + 1024;
  for (int side = 0; side < 2; ++side) {
    const int site = side == 0 ? si : sj, leg = side == 0 ? li : lj;
    const double* w0 = wptr(site, other_leg(leg, 0));
    const double* w1 = wptr(site, other_leg(leg, 1));
    const double* w2 = wptr(site, other_leg(leg, 2));
    const long s0 = leg_stride(other_leg(leg, 0), D, d), s1 = leg_stride(other_leg(leg, 1), D, d);
    const long s2 = leg_stride(other_leg(leg, 2), D, d), sb = leg_stride(leg, D, d);
    const T* Gs = G + (long)site * T_;
    for (long e = tid; e < (long)R * C; e += 256) {
      const int r = (int)(e / C), c = (int)(e % C);
      const int a1 = r / (D * D), a2 = (r / D) % D, a3 = r % D, kk = c / d, p = c % d;
      A[e] = Gs[a1 * s0 + a2 * s1 + a3 * s2 + kk * sb + p] * (w0[a1] * w1[a2] * w2[a3]);
    }
    __syncthreads();
    T* K = side == 0 ? Ki : Kj;
    for (int e = tid; e < C * C; e += 256) {
      const int c1 = e / C, c2 = e % C;
      T acc = szero<T>();
      for (int r = 0; r < R; ++r) acc += cmul(A[(long)r * C + c2], A[(long)r * C + c1]);
      K[e] = acc;
    }
    __syncthreads();
  }
  // rho[(p q)][(p' q')] = sum_{k k'} Ki[(k p)][(k' p')] lam_k lam_k' Kj[(k q)][(k' q')]
  const int n4 = d2 * d2;
  for (int e = tid; e < n4; e += 256) {
    const int row = e / d2, col = e % d2;
    const int p = row / d, q = row % d, p2 = col / d, q2 = col % d;
    T acc = szero<T>();
    for (int k1 = 0; k1 < D; ++k1)
      for (int k2 = 0; k2 < D; ++k2)
        acc += Ki[(k1 * d + p) * C + k2 * d + p2] * Kj[(k1 * d + q) * C + k2 * d + q2] * (lamB[k1] * lamB[k2]);
    red[e] = acc;
  }
  __syncthreads();
  if (tid < n4) {
    double tr = 0.0;
    for (int a = 0; a < d2; ++a) tr += sre(red[a * d2 + a]);
    rho2[(((long)b * N + s) * 2 + dir) * n4 + tid] = red[tid] * (1.0 / tr);
  }
}

// energy[b] = (1/N) sum_s (sum_dir tr(rho2 H) + tr(rho1 onsite)), each
// expectation the real part of sum rho[in][out] O[out][in] of unit-trace
// density matrices.
template <typename T>
__global__ __launch_bounds__(256) void k_su_energy(const double* rho1d, const double* rho2d, const double* Hd,
                                                   const double* onsited, double* energy, double* bond_e, int N, int d) {
  __shared__ double red[256];
  const T* rho1 = reinterpret_cast<const T*>(rho1d);
  const T* rho2 = reinterpret_cast<const T*>(rho2d);
  const T* H = reinterpret_cast<const T*>(Hd);
  const T* onsite = reinterpret_cast<const T*>(onsited);
  const int b = blockIdx.x, tid = threadIdx.x, d2 = d * d, n4 = d2 * d2;
  double acc = 0.0;
  for (int s = 0; s < N; ++s) {
    for (int dir = 0; dir < 2; ++dir) {
      const long base = (((long)b * N + s) * 2 + dir) * n4;
      double part = 0.0;
      for (int e = tid; e < n4; e += 256) {
        const int a = e / d2, c = e % d2;
        part += sre(rho2[base + e] * H[base + (long)c * d2 + a]);
      }
      red[tid] = part;
      __syncthreads();
      for (int h = 128; h >= 1; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
      }
      if (tid == 0) {
        acc += red[0];
        if (bond_e) bond_e[((long)b * N + s) * 2 + dir] = red[0];
      }
      __syncthreads();
    }
    if (onsite && tid == 0) {
      const T* r1 = rho1 + ((long)b * N + s) * d2;
      const T* o = onsite + (long)b * d2;
      for (int a = 0; a < d; ++a)
        for (int c = 0; c < d; ++c) acc += sre(r1[a * d + c] * o[c * d + a]);
    }
  }
  if (tid == 0) energy[b] = acc / N;
}

// A_s = G_s with sqrt(weight) on every leg (the iTPS the state stands for).
template <typename T>
__global__ void k_su_itps(const double* gammad, const double* lam, double* outd, int Lx, int Ly, int D, int d,
                          long total) {
  const T* gamma = reinterpret_cast<const T*>(gammad);
  T* out = reinterpret_cast<T*>(outd);
  const int N = Lx * Ly;
  const long T_ = (long)D * D * D * D * d;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long bs = e / T_, r = e % T_;
    const int b = (int)(bs / N), s = (int)(bs % N);
    const int l = (int)(r / ((long)D * D * D * d)), u = (int)((r / ((long)D * D * d)) % D);
    const int rr = (int)((r / ((long)D * d)) % D), dd = (int)((r / d) % D);
    const double* lamL = lam + (long)b * N * 2 * D;
    const int sx = s % Lx, sy = s / Lx;
    const double wl = lamL[(((sx - 1 + Lx) % Lx + Lx * sy) * 2 + 0) * D + l];
    const double wu = lamL[(s * 2 + 1) * D + u];
    const double wr = lamL[(s * 2 + 0) * D + rr];
    const double wd = lamL[((sx + Lx * ((sy - 1 + Ly) % Ly)) * 2 + 1) * D + dd];
    out[e] = gamma[e] * sqrt(wl * wu * wr * wd);
  }
}

}  // namespace

void trotter_gates(hipStream_t st, const double* H, const double* tau, double* gates, int N, int d2, int batch) {
  hipLaunchKernelGGL(k_su_gates<double>, dim3(batch * N * 2), dim3(256), 0, st, H, tau, gates, N, d2);
  CTM_HIP(hipGetLastError());
}

}  // namespace ctm

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
struct ctm_su {
  ctm_su_config cfg{};
  ctm::SuShape S{};
  hipStream_t st = nullptr;
  bool own_stream = false;
  int cap = 0;                // index of the kernel instantiation
  bool cplx = false;          // complex tensors and Hamiltonians
  int words = 1;              // doubles per scalar (1 real, 2 complex)
  ctm::DevBuf gamma, lam, H, tau, gates, status, rho1, rho2, energy, bond_e, onsite;
  bool gates_set = false;
  double last_ms = 0.0;
  long last_launches = 0;
  long bond_updates = 0;
  std::string err;
};

namespace {

thread_local std::string g_su_static_err;

template <typename F>
ctm_status su_guarded(ctm_su* su, F&& f) {
  try {
    f();
    return CTM_OK;
  } catch (const ctm::Error& e) {
    if (su) su->err = e.what();
    else g_su_static_err = e.what();
    return (ctm_status)e.status;
  } catch (const std::bad_alloc&) {
    if (su) su->err = "host allocation failed";
    return CTM_ENOMEM;
  } catch (const std::exception& e) {
    if (su) su->err = e.what();
    else g_su_static_err = e.what();
    return CTM_EDEVICE;
  }
}

// kernel instantiations: (scalar, LDS doubles, rows per lane, columns per wave)
struct SuKernelClass {
  bool cplx;
  int cap, rpl, cpw;
  void (*fn)(ctm::SuArgs);
};
const SuKernelClass kSuClasses[] = {
    {false, 3072, 1, 2, ctm::k_su_run<double, 3072, 1, 2>},   {false, 3072, 1, 4, ctm::k_su_run<double, 3072, 1, 4>},
    {false, 8192, 2, 4, ctm::k_su_run<double, 8192, 2, 4>},   {false, 8192, 4, 8, ctm::k_su_run<double, 8192, 4, 8>},
    {false, 20224, 4, 8, ctm::k_su_run<double, 20224, 4, 8>}, {false, 20224, 8, 8, ctm::k_su_run<double, 20224, 8, 8>},
    {true, 3072, 1, 2, ctm::k_su_run<ctm::zc, 3072, 1, 2>},   {true, 8192, 1, 4, ctm::k_su_run<ctm::zc, 8192, 1, 4>},
    {true, 8192, 2, 4, ctm::k_su_run<ctm::zc, 8192, 2, 4>},   {true, 20224, 4, 8, ctm::k_su_run<ctm::zc, 20224, 4, 8>},
};

// the smallest instantiation that holds the shape, or -1
int su_kernel_class(const ctm::SuShape& S, bool cplx) {
  const long need = ctm::su_lds_need(S, cplx ? 2 : 1);
  const int rpl = (S.R + 63) / 64, cpw = (S.C + ctm::kSuWaves - 1) / ctm::kSuWaves;
  for (int i = 0; i < (int)(sizeof(kSuClasses) / sizeof(kSuClasses[0])); ++i)
    if (kSuClasses[i].cplx == cplx && need <= kSuClasses[i].cap && rpl <= kSuClasses[i].rpl &&
        cpw <= kSuClasses[i].cpw)
      return i;
  return -1;
}

void su_launch_mfe(ctm_su* su) {
  const dim3 grid(su->S.N, 3, su->cfg.batch);
  if (su->cplx)
    hipLaunchKernelGGL(ctm::k_su_mfe<ctm::zc>, grid, dim3(256), 0, su->st, su->gamma.as<double>(),
                       su->lam.as<double>(), su->rho1.as<double>(), su->rho2.as<double>(), su->cfg.Lx, su->cfg.Ly,
                       su->cfg.D, su->cfg.d);
  else
    hipLaunchKernelGGL(ctm::k_su_mfe<double>, grid, dim3(256), 0, su->st, su->gamma.as<double>(),
                       su->lam.as<double>(), su->rho1.as<double>(), su->rho2.as<double>(), su->cfg.Lx, su->cfg.Ly,
                       su->cfg.D, su->cfg.d);
}

void su_launch_run(ctm_su* su, int nsteps) {
  ctm::SuArgs a;
  a.gamma = su->gamma.as<double>();
  a.lam = su->lam.as<double>();
  a.gates = su->gates.as<double>();
  a.status = su->status.as<int>();
  a.Lx = su->cfg.Lx; a.Ly = su->cfg.Ly; a.D = su->cfg.D; a.d = su->cfg.d; a.nsteps = nsteps;
  hipLaunchKernelGGL(kSuClasses[su->cap].fn, dim3(su->cfg.batch), dim3(ctm::kSuThreads), 0, su->st, a);
  CTM_HIP(hipGetLastError());
}

}  // namespace

extern "C" {

ctm_status ctm_su_create(const ctm_su_config* cfg, const double* gamma, const double* lambda, ctm_su** out) {
  if (out) *out = nullptr;
  return su_guarded(nullptr, [&] {
    CTM_CHECK(cfg && gamma && lambda && out, CTM_EINVAL, "NULL argument");
    CTM_CHECK(cfg->Lx >= 2 && cfg->Ly >= 2 && cfg->Lx * cfg->Ly <= 16, CTM_EINVAL,
              "the simple update needs Lx >= 2, Ly >= 2 and at most 16 sites");
    CTM_CHECK(cfg->D >= 1 && cfg->D <= 8, CTM_EINVAL, "D must be in 1..8");
    CTM_CHECK(cfg->d >= 1 && cfg->d <= 4, CTM_EINVAL, "d must be in 1..4");
    CTM_CHECK(cfg->batch >= 1 && cfg->batch <= 65535, CTM_EINVAL, "batch must be in 1..65535");
    const ctm::SuShape S = ctm::su_shape(cfg->Lx, cfg->Ly, cfg->D, cfg->d);
    CTM_CHECK(S.m <= 64, CTM_EINVAL, "min(D^3, D d) * d must be <= 64");
    CTM_CHECK(cfg->complex_tensors == 0 || cfg->complex_tensors == 1, CTM_EINVAL, "complex_tensors must be 0 or 1");
    const bool cplx = cfg->complex_tensors == 1;
    const int words = cplx ? 2 : 1;
    const int cap = su_kernel_class(S, cplx);
    CTM_CHECK(cap >= 0, CTM_EINVAL, "bond tensors too large for one workgroup's LDS");
    CTM_CHECK((long)S.R * S.C <= (cplx ? ctm::mfe_a_cap<ctm::zc>() : ctm::mfe_a_cap<double>()) && S.C <= 32,
              CTM_EINVAL, "bond tensors too large for the mean-field kernel's LDS");
    {
      const long B = cfg->batch, T = (long)S.N * S.R * S.D * S.d * words, L = (long)S.N * 2 * S.D;
      for (long e = 0; e < B * T; ++e) CTM_CHECK(std::isfinite(gamma[e]), CTM_EINVAL, "site tensors must be finite");
      for (long e = 0; e < B * L; ++e)
        CTM_CHECK(std::isfinite(lambda[e]) && lambda[e] >= 0.0, CTM_EINVAL, "bond weights must be finite and >= 0");
    }
    auto su = new ctm_su();
    try {
      su->cfg = *cfg;
      su->S = S;
      su->cap = cap;
      su->cplx = cplx;
      su->words = words;
      if (cfg->stream) {
        su->st = (hipStream_t)cfg->stream;
      } else {
        CTM_HIP(hipStreamCreateWithFlags(&su->st, hipStreamNonBlocking));
        su->own_stream = true;
      }
      const long B = cfg->batch, N = S.N, T = (long)S.R * S.D * S.d, n4 = (long)S.d2 * S.d2, w = words;
      su->gamma.alloc(B * N * T * w * sizeof(double));
      su->lam.alloc(B * N * 2 * S.D * sizeof(double));
      su->H.alloc(B * N * 2 * n4 * w * sizeof(double));
      su->tau.alloc(B * sizeof(double));
      su->gates.alloc(B * N * 2 * n4 * w * sizeof(double));
      su->status.alloc(B * sizeof(int));
      su->rho1.alloc(B * N * S.d2 * w * sizeof(double));
      su->rho2.alloc(B * N * 2 * n4 * w * sizeof(double));
      su->energy.alloc(B * sizeof(double));
      su->bond_e.alloc(B * N * 2 * sizeof(double));
      su->onsite.alloc(B * S.d2 * w * sizeof(double));
      CTM_HIP(hipMemcpyAsync(su->gamma.p, gamma, su->gamma.bytes, hipMemcpyHostToDevice, su->st));
      CTM_HIP(hipMemcpyAsync(su->lam.p, lambda, su->lam.bytes, hipMemcpyHostToDevice, su->st));
      CTM_HIP(hipMemsetAsync(su->status.p, 0, su->status.bytes, su->st));
      CTM_HIP(hipStreamSynchronize(su->st));
    } catch (...) {
      if (su->own_stream && su->st) (void)hipStreamDestroy(su->st);
      delete su;
      throw;
    }
    *out = su;
  });
}

ctm_status ctm_su_set_hamiltonians(ctm_su* su, const double* H, const double* tau) {
  if (!su) return CTM_EINVAL;
  return su_guarded(su, [&] {
    CTM_CHECK(H && tau, CTM_EINVAL, "NULL argument");
    const long B = su->cfg.batch;
    for (long b = 0; b < B; ++b) CTM_CHECK(std::isfinite(tau[b]) && tau[b] >= 0.0, CTM_EINVAL, "tau must be finite and >= 0");
    const long n = (long)su->S.N * 2 * su->S.d2 * su->S.d2 * su->words;
    for (long e = 0; e < B * n; ++e) CTM_CHECK(std::isfinite(H[e]), CTM_EINVAL, "Hamiltonian entries must be finite");
    CTM_HIP(hipMemcpyAsync(su->H.p, H, su->H.bytes, hipMemcpyHostToDevice, su->st));
    CTM_HIP(hipMemcpyAsync(su->tau.p, tau, su->tau.bytes, hipMemcpyHostToDevice, su->st));
    if (su->cplx)
      hipLaunchKernelGGL(ctm::k_su_gates<ctm::zc>, dim3(B * su->S.N * 2), dim3(256), 0, su->st, su->H.as<double>(),
                         su->tau.as<double>(), su->gates.as<double>(), su->S.N, su->S.d2);
    else
      hipLaunchKernelGGL(ctm::k_su_gates<double>, dim3(B * su->S.N * 2), dim3(256), 0, su->st, su->H.as<double>(),
                         su->tau.as<double>(), su->gates.as<double>(), su->S.N, su->S.d2);
    CTM_HIP(hipGetLastError());
    CTM_HIP(hipStreamSynchronize(su->st));
    su->gates_set = true;
  });
}

ctm_status ctm_su_run(ctm_su* su, int nsteps) {
  if (!su) return CTM_EINVAL;
  return su_guarded(su, [&] {
    CTM_CHECK(nsteps >= 0, CTM_EINVAL, "nsteps must be >= 0");
    CTM_CHECK(su->gates_set, CTM_EINVAL, "ctm_su_set_hamiltonians has not been called");
    hipEvent_t e0, e1;
    CTM_HIP(hipEventCreate(&e0));
    CTM_HIP(hipEventCreate(&e1));
    long launches = 0;
    try {
      CTM_HIP(hipMemsetAsync(su->status.p, 0, su->status.bytes, su->st));
      CTM_HIP(hipEventRecord(e0, su->st));
      for (int done = 0; done < nsteps; done += ctm::kSuStepsPerLaunch) {
        su_launch_run(su, std::min(ctm::kSuStepsPerLaunch, nsteps - done));
        ++launches;
      }
      CTM_HIP(hipEventRecord(e1, su->st));
      CTM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      CTM_HIP(hipEventElapsedTime(&ms, e0, e1));
      su->last_ms = ms;
      su->last_launches = launches;
      su->bond_updates = (long)nsteps * 2 * su->S.N * su->cfg.batch;
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::vector<int> stv(su->cfg.batch);
    CTM_HIP(hipMemcpy(stv.data(), su->status.p, su->status.bytes, hipMemcpyDeviceToHost));
    for (int b = 0; b < su->cfg.batch; ++b)
      CTM_CHECK(stv[b] == 0, CTM_ENUMERIC, "problem " + std::to_string(b) +
                                               ": a bond lost every singular value (zero or non-finite state)");
  });
}

ctm_status ctm_su_stats(const ctm_su* su, double* gpu_ms, long* launches, long* bond_updates) {
  if (!su) return CTM_EINVAL;
  if (gpu_ms) *gpu_ms = su->last_ms;
  if (launches) *launches = su->last_launches;
  if (bond_updates) *bond_updates = su->bond_updates;
  return CTM_OK;
}

ctm_status ctm_su_get(ctm_su* su, double* gamma, double* lambda) {
  if (!su) return CTM_EINVAL;
  return su_guarded(su, [&] {
    if (gamma) CTM_HIP(hipMemcpyAsync(gamma, su->gamma.p, su->gamma.bytes, hipMemcpyDeviceToHost, su->st));
    if (lambda) CTM_HIP(hipMemcpyAsync(lambda, su->lam.p, su->lam.bytes, hipMemcpyDeviceToHost, su->st));
    CTM_HIP(hipStreamSynchronize(su->st));
  });
}

ctm_status ctm_su_get_itps(ctm_su* su, double* tensors, int on_device) {
  if (!su) return CTM_EINVAL;
  return su_guarded(su, [&] {
    CTM_CHECK(tensors, CTM_EINVAL, "NULL argument");
    const long total = (long)su->cfg.batch * su->S.N * su->S.R * su->S.D * su->S.d;
    const long bytes = total * su->words * (long)sizeof(double);
    ctm::DevBuf tmp;
    double* dst = tensors;
    if (!on_device) {
      tmp.alloc(bytes);
      dst = tmp.as<double>();
    }
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    if (su->cplx)
      hipLaunchKernelGGL(ctm::k_su_itps<ctm::zc>, dim3(blocks), dim3(256), 0, su->st, su->gamma.as<double>(),
                         su->lam.as<double>(), dst, su->cfg.Lx, su->cfg.Ly, su->cfg.D, su->cfg.d, total);
    else
      hipLaunchKernelGGL(ctm::k_su_itps<double>, dim3(blocks), dim3(256), 0, su->st, su->gamma.as<double>(),
                         su->lam.as<double>(), dst, su->cfg.Lx, su->cfg.Ly, su->cfg.D, su->cfg.d, total);
    CTM_HIP(hipGetLastError());
    if (!on_device) CTM_HIP(hipMemcpyAsync(tensors, dst, bytes, hipMemcpyDeviceToHost, su->st));
    CTM_HIP(hipStreamSynchronize(su->st));
  });
}

ctm_status ctm_su_mfe(ctm_su* su, double* rho1, double* rho2) {
  if (!su) return CTM_EINVAL;
  return su_guarded(su, [&] {
    su_launch_mfe(su);
    CTM_HIP(hipGetLastError());
    if (rho1) CTM_HIP(hipMemcpyAsync(rho1, su->rho1.p, su->rho1.bytes, hipMemcpyDeviceToHost, su->st));
    if (rho2) CTM_HIP(hipMemcpyAsync(rho2, su->rho2.p, su->rho2.bytes, hipMemcpyDeviceToHost, su->st));
    CTM_HIP(hipStreamSynchronize(su->st));
  });
}

ctm_status ctm_su_mfe_energy(ctm_su* su, const double* onsite, double* energy, double* bond_energy) {
  if (!su) return CTM_EINVAL;
  return su_guarded(su, [&] {
    CTM_CHECK(energy, CTM_EINVAL, "NULL argument");
    CTM_CHECK(su->gates_set, CTM_EINVAL, "ctm_su_set_hamiltonians has not been called");
    if (onsite) CTM_HIP(hipMemcpyAsync(su->onsite.p, onsite, su->onsite.bytes, hipMemcpyHostToDevice, su->st));
    su_launch_mfe(su);
    CTM_HIP(hipGetLastError());
    if (su->cplx)
      hipLaunchKernelGGL(ctm::k_su_energy<ctm::zc>, dim3(su->cfg.batch), dim3(256), 0, su->st, su->rho1.as<double>(),
                         su->rho2.as<double>(), su->H.as<double>(), onsite ? su->onsite.as<double>() : nullptr,
                         su->energy.as<double>(), su->bond_e.as<double>(), su->S.N, su->cfg.d);
    else
      hipLaunchKernelGGL(ctm::k_su_energy<double>, dim3(su->cfg.batch), dim3(256), 0, su->st, su->rho1.as<double>(),
                         su->rho2.as<double>(), su->H.as<double>(), onsite ? su->onsite.as<double>() : nullptr,
                         su->energy.as<double>(), su->bond_e.as<double>(), su->S.N, su->cfg.d);
    CTM_HIP(hipGetLastError());
    CTM_HIP(hipMemcpyAsync(energy, su->energy.p, su->energy.bytes, hipMemcpyDeviceToHost, su->st));
    if (bond_energy)
      CTM_HIP(hipMemcpyAsync(bond_energy, su->bond_e.p, su->bond_e.bytes, hipMemcpyDeviceToHost, su->st));
    CTM_HIP(hipStreamSynchronize(su->st));
  });
}

const char* ctm_su_last_error(const ctm_su* su) {
  if (!su) return g_su_static_err.empty() ? "null simple-update handle" : g_su_static_err.c_str();
  return su->err.c_str();
}

void ctm_su_free(ctm_su* su) {
  if (!su) return;
  if (su->st) (void)hipStreamSynchronize(su->st);
  const bool own = su->own_stream;
  hipStream_t st = su->st;
  delete su;
  if (own && st) (void)hipStreamDestroy(st);
}

}  // extern "C"
