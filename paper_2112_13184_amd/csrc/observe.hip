// Expectation values from the converged environment (Sec. 5.3 of arXiv:2112.13184).
//
// Each quantity is a ratio of contractions of one finite patch (3x3 for one
// site, 3x4 / 4x3 for a bond), so the normalisation of C and T drops out.  The
// patch is contracted column by column: left boundary LB[t1][l][t3] = C1 T4 C4,
// one column per site (T1 above, ket then bra site tensor, T3 below), right
// boundary RB[t1][r][t3] = C2 T2 C3.  Contractions are permute + MFMA GEMM
// (tensordot) on transient buffers; all of it runs once per solve.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "context.hpp"
#include "hessenberg.hpp"
#include "kernels.hpp"

namespace ctm {
namespace {

inline int mod(int a, int b) { return ((a % b) + b) % b; }

int view_site(const Context& c, int rot, int xv, int yv) {
  int x = xv, y = yv;
  for (int i = 0; i < rot; ++i) { int t = x; x = y; y = -t; }
  return mod(x, c.Lx) + c.Lx * mod(y, c.Ly);
}

DT make(double* p, std::vector<long> dims) { DT t; t.p = p; t.dims = std::move(dims); return t; }

DT transpose(Context& c, const DT& A, const std::vector<int>& perm) {
  bool ident = true;
  for (size_t i = 0; i < perm.size(); ++i) ident &= (perm[i] == (int)i);
  if (ident) return A;
  DT out;
  out.dims.resize(perm.size());
  for (size_t i = 0; i < perm.size(); ++i) out.dims[i] = A.dims[perm[i]];
  out.p = c.arena.alloc(A.size());
  permute(c.st, A.p, out.p, (int)A.dims.size(), A.dims.data(), perm.data());
  return out;
}

// numpy.tensordot(A, B, axes=(axA, axB)): free axes of A, then free axes of B.
DT tdot(Context& c, const DT& A, const std::vector<int>& axA, const DT& B, const std::vector<int>& axB) {
  std::vector<int> fa, fb;
  for (int i = 0; i < (int)A.dims.size(); ++i)
    if (std::find(axA.begin(), axA.end(), i) == axA.end()) fa.push_back(i);
  for (int i = 0; i < (int)B.dims.size(); ++i)
    if (std::find(axB.begin(), axB.end(), i) == axB.end()) fb.push_back(i);
  std::vector<int> pa = fa, pb = axB;
  pa.insert(pa.end(), axA.begin(), axA.end());
  pb.insert(pb.end(), fb.begin(), fb.end());
  DT Ap = transpose(c, A, pa), Bp = transpose(c, B, pb);
  long M = 1, K = 1, N = 1;
  std::vector<long> od;
  for (int i : fa) { M *= A.dims[i]; od.push_back(A.dims[i]); }
  for (size_t i = 0; i < axA.size(); ++i) {
    CTM_CHECK(A.dims[axA[i]] == B.dims[axB[i]], -1, "tdot: contracted dims differ");
    K *= A.dims[axA[i]];
  }
  for (int i : fb) { N *= B.dims[i]; od.push_back(B.dims[i]); }
  DT out;
  out.dims = od;
  out.p = c.arena.alloc((size_t)std::max<long>(M * N, 1));
  gemm(c.st, GemmType::F64, (int)M, (int)N, (int)K, 1.0, rowmajor(Ap.p, K), rowmajor(Bp.p, N), 0.0,
       out_rowmajor(out.p, N), 1, c.ws());
  return out;
}

struct View {
  DT C[4], T[4], Ak, Ab;
};

View view_of(Context& c, int s, int rot) {
  View v;
  const long chi = c.chi, Db = c.Db;
  for (int m = 0; m < 4; ++m) {
    v.C[m] = make(c.C(s, (m + rot) % 4), {chi, chi});
    v.T[m] = make(c.Ta(s, (m + rot) % 4), {chi, chi, Db});
  }
  v.Ak = make(const_cast<double*>(c.Ak(rot, s)), {c.DK, c.DK, c.DK, c.DK, c.d});
  v.Ab = make(const_cast<double*>(c.Ab(rot, s)), {c.DB, c.DB, c.DB, c.DB, c.d});
  return v;
}

DT left_boundary(Context& c, const View& v) {
  DT X = tdot(c, v.C[0], {1}, v.T[3], {1});     // C1[t1][a] T4[b][a][l] -> [t1][b][l]
  return tdot(c, X, {1}, v.C[3], {0});           // C4[b][t3] -> [t1][l][t3]
}

DT right_boundary(Context& c, const View& v) {
  DT X = tdot(c, v.C[1], {0}, v.T[1], {0});     // C2[a][t1] T2[a][b][r] -> [t1][b][r]
  return tdot(c, X, {1}, v.C[2], {1});           // C3[t3][b] -> [t1][r][t3]
}

// LB[t1][Lp][t3][e...] through the column of one site; open: append (p, p').
DT column(Context& c, const DT& LB, const DT& T1, const DT& T3, const DT& Ak, const DT& Ab, bool open) {
  const int ne = (int)LB.dims.size() - 3;
  const long DK = c.DK, DB = c.DB;
  DT X = tdot(c, LB, {0}, T1, {0});              // [Lp, t3, e.., t1', U]
  std::vector<long> xd = {DK, DB};
  for (int i = 1; i < (int)X.dims.size() - 1; ++i) xd.push_back(X.dims[i]);
  xd.push_back(DK);
  xd.push_back(DB);
  X.dims = xd;                                   // [Lk, Lb, t3, e.., t1', Uk, Ub]
  DT Y = tdot(c, X, {0, 4 + ne}, Ak, {0, 1});    // [Lb, t3, e.., t1', Ub, Rk, Dk, p]
  DT Z;
  std::vector<int> perm;
  if (!open) {
    Z = tdot(c, Y, {0, 3 + ne, 6 + ne}, Ab, {0, 1, 4});   // [t3, e.., t1', Rk, Dk, Rb, Db]
    perm = {1 + ne, 2 + ne, 4 + ne, 0, 3 + ne, 5 + ne};
    for (int i = 1; i <= ne; ++i) perm.push_back(i);
  } else {
    Z = tdot(c, Y, {0, 3 + ne}, Ab, {0, 1});              // [t3, e.., t1', Rk, Dk, p, Rb, Db, p']
    perm = {1 + ne, 2 + ne, 5 + ne, 0, 3 + ne, 6 + ne};
    for (int i = 1; i <= ne; ++i) perm.push_back(i);
    perm.push_back(4 + ne);
    perm.push_back(7 + ne);
  }
  Z = transpose(c, Z, perm);                     // [t1', Rk, Rb, t3, Dk, Db, e.., (p, p')]
  std::vector<long> zd = {Z.dims[0], DK * DB, Z.dims[3], DK * DB};
  for (size_t i = 6; i < Z.dims.size(); ++i) zd.push_back(Z.dims[i]);
  Z.dims = zd;                                   // [t1', R, t3, Dd, e.., (p, p')]
  DT W = tdot(c, Z, {2, 3}, T3, {1, 2});         // [t1', R, e.., (p, p'), t3']
  std::vector<int> p2 = {0, 1, (int)W.dims.size() - 1};
  for (int i = 2; i < (int)W.dims.size() - 1; ++i) p2.push_back(i);
  return transpose(c, W, p2);                    // [t1', R, t3', e.., (p, p')]
}

DT close_lr(Context& c, const DT& X, const DT& RB) { return tdot(c, X, {0, 1, 2}, RB, {0, 1, 2}); }

__global__ void k_trace_normalize(const double* in, double* out, int dim) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < dim; ++i) tr += in[i * dim + i];
    for (int i = 0; i < dim * dim; ++i) out[i] = in[i] / tr;
  }
}

__global__ void k_expect(const double* rho, const double* op, int dim, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < dim; ++i)
      for (int o = 0; o < dim; ++o) s += rho[i * dim + o] * op[o * dim + i];
    *out = s;
  }
}

// ln |z33 zc / (z23 z32)| and z_b / z_a
__global__ void k_logkappa(const double* z33, const double* zc, const double* z23, const double* z32, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = log(fabs(*z33)) + log(fabs(*zc)) - log(fabs(*z23)) - log(fabs(*z32));
}
__global__ void k_ratio(const double* a, const double* b, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = *a / *b;
}

double fetch_scalar(Context& c, const double* dev) {
  double h = 0.0;
  d2h(c, &h, dev, 1);
  return h;
}

}  // namespace

DT tensordot(Context& c, const DT& A, const std::vector<int>& axA, const DT& B, const std::vector<int>& axB) {
  return tdot(c, A, axA, B, axB);
}

DT tensor_transpose(Context& c, const DT& A, const std::vector<int>& perm) { return transpose(c, A, perm); }

// B = A / tr(A), A dim x dim: one workgroup
__global__ __launch_bounds__(256) void k_trace_scale(const double* A, double* B, int dim) {
  __shared__ double red[256];
  double t = 0.0;
  for (int i = threadIdx.x; i < dim; i += 256) t += A[(long)i * dim + i];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double inv = 1.0 / red[0];
  for (long e = threadIdx.x; e < (long)dim * dim; e += 256) B[e] = A[e] * inv;
}

DT bond_environment(Context& c, int site, int dir, const double* Ei, const double* Ej, int r) {
  const int rot = (dir == 0) ? 0 : 3;   // +y becomes +x three quarter turns on
  int x = site % c.Lx, y = site / c.Lx;
  for (int i = 0; i < rot; ++i) { int t = x; x = -y; y = t; }
  const int s = view_site(c, rot, x, y), t = view_site(c, rot, x + 1, y);
  CTM_CHECK(s == site, -3, "bond_environment: view bookkeeping");
  // The left half (C1 T4 C4, T1 / X_i / T3 of site s) in the frame `rot`, the
  // right half as a left half of site t in the frame turned two more quarter
  // turns (there C3 T2 C2 form its left boundary and T3 / T1 sit above /
  // below); the two meet on the cut bond and on the edge legs between the
  // columns, so neither half carries the other's open legs.
  const int rot2 = (rot + 2) % 4;
  View vs = view_of(c, s, rot), vt = view_of(c, t, rot2);
  const long D = c.D;
  DT ei = make(const_cast<double*>(Ei), {D, D, D, D, (long)r});
  DT ej = make(const_cast<double*>(Ej), {D, D, D, D, (long)r});
  for (int q = 0; q < rot; ++q) ei = transpose(c, ei, {1, 2, 3, 0, 4});    // a quarter turn each
  for (int q = 0; q < rot2; ++q) ej = transpose(c, ej, {1, 2, 3, 0, 4});
  DT Xi = column(c, left_boundary(c, vs), vs.T[0], vs.T[2], ei, ei, true);   // [t1', R, t3', ri, ri']
  DT Xj = column(c, left_boundary(c, vt), vt.T[0], vt.T[2], ej, ej, true);   // [t3-side, R, t1-side, rj, rj']
  // Xi's t1' (right leg of T1 of s) meets the leg of T1 of t that Xj leaves
  // as its third index, Xi's t3' its first
  DT R = tdot(c, Xi, {0, 1, 2}, Xj, {2, 1, 0});   // [ri, ri', rj, rj']
  R = transpose(c, R, {0, 2, 1, 3});             // [(ri, rj), (ri', rj')]
  const int dim = r * r;
  DT N = make(c.arena.alloc((size_t)dim * dim), {(long)dim, (long)dim});
  hipLaunchKernelGGL(k_trace_scale, dim3(1), dim3(256), 0, c.st, R.p, N.p, dim);
  CTM_HIP(hipGetLastError());
  return N;
}

void rho_1site(Context& c, int site, double* rho_dev, double* rho_host) {
  c.arena.reset();
  View v = view_of(c, site, 0);
  DT LB = left_boundary(c, v), RB = right_boundary(c, v);
  DT X = column(c, LB, v.T[0], v.T[2], v.Ak, v.Ab, true);
  DT R = close_lr(c, X, RB);                     // [p, p']
  hipLaunchKernelGGL(k_trace_normalize, dim3(1), dim3(64), 0, c.st, R.p, rho_dev, c.d);
  CTM_HIP(hipGetLastError());
  if (rho_host) {
    CTM_HIP(hipMemcpyAsync(rho_host, rho_dev, sizeof(double) * c.d * c.d, hipMemcpyDeviceToHost, c.st));
    CTM_HIP(hipStreamSynchronize(c.st));
  }
}

void rho_2site(Context& c, int site, int dir, double* rho_dev, double* rho_host) {
  c.arena.reset();
  const int rot = (dir == 0) ? 0 : 3;   // +y becomes +x three quarter turns on
  int x = site % c.Lx, y = site / c.Lx;
  for (int i = 0; i < rot; ++i) { int t = x; x = -y; y = t; }
  const int s = view_site(c, rot, x, y), t = view_site(c, rot, x + 1, y);
  CTM_CHECK(s == site, -3, "rho_2site: view bookkeeping");
  View vs = view_of(c, s, rot), vt = view_of(c, t, rot);
  DT LB = left_boundary(c, vs), RB = right_boundary(c, vt);
  DT X = column(c, LB, vs.T[0], vs.T[2], vs.Ak, vs.Ab, true);
  X = column(c, X, vt.T[0], vt.T[2], vt.Ak, vt.Ab, true);
  DT R = close_lr(c, X, RB);                     // [ps, ps', pt, pt']
  R = transpose(c, R, {0, 2, 1, 3});             // [(ps, pt), (ps', pt')]
  const int dim = c.d * c.d;
  hipLaunchKernelGGL(k_trace_normalize, dim3(1), dim3(64), 0, c.st, R.p, rho_dev, dim);
  CTM_HIP(hipGetLastError());
  if (rho_host) {
    CTM_HIP(hipMemcpyAsync(rho_host, rho_dev, sizeof(double) * dim * dim, hipMemcpyDeviceToHost, c.st));
    CTM_HIP(hipStreamSynchronize(c.st));
  }
}

namespace {

// The bra tensor with a one-site operator on its physical leg,
// AbO[l,u,r,d,p] = sum_p' O[p'][p] Ab[l,u,r,d,p'], so that the closed
// contraction sum_p A[..p] AbO[..p] equals sum_{p,p'} A[..p] O[p'][p] A*[..p'].
DT bra_with_op(Context& c, const DT& Ab, const double* op_host) {
  const int d = c.d;
  double* o = c.arena.alloc((size_t)d * d);
  CTM_HIP(hipMemcpyAsync(o, op_host, sizeof(double) * d * d, hipMemcpyHostToDevice, c.st));
  DT out;
  out.dims = Ab.dims;
  out.p = c.arena.alloc(Ab.size());
  gemm(c.st, GemmType::F64, (int)(Ab.size() / d), d, d, 1.0, rowmajor(Ab.p, d), rowmajor(o, d), 0.0,
       out_rowmajor(out.p, d), 1, c.ws());
  return out;
}

void keep(Context& c, const DT& src, double* dst) {
  CTM_HIP(hipMemcpyAsync(dst, src.p, sizeof(double) * src.size(), hipMemcpyDeviceToDevice, c.st));
}

std::vector<double> fetch(Context& c, const double* dev, size_t n) {
  std::vector<double> h(n);
  d2h(c, h.data(), dev, n);
  return h;
}

}  // namespace

double expect_1site(Context& c, int site, const double* op_host, int replica) {
  c.arena.reset();
  View v = view_of(c, replica * c.N + site, 0);
  double* res = c.arena.alloc(2);   // value with the operator, norm
  DT LB = left_boundary(c, v), RB = right_boundary(c, v);
  const auto m = c.arena.mark();
  for (int t = 0; t < 2; ++t) {
    DT Ab = (t == 0) ? bra_with_op(c, v.Ab, op_host) : v.Ab;
    keep(c, close_lr(c, column(c, LB, v.T[0], v.T[2], v.Ak, Ab, false), RB), res + t);
    c.arena.release(m);
  }
  const std::vector<double> h = fetch(c, res, 2);
  return h[0] / h[1];
}

double expect_2site(Context& c, int site, int dir, const double* op_host, int replica) {
  c.arena.reset();
  const int rot = (dir == 0) ? 0 : 3;
  int x = site % c.Lx, y = site / c.Lx;
  for (int i = 0; i < rot; ++i) { int t = x; x = -y; y = t; }
  const int s = view_site(c, rot, x, y), t = view_site(c, rot, x + 1, y);
  CTM_CHECK(s == site, -3, "expect_2site: view bookkeeping");
  View vs = view_of(c, replica * c.N + s, rot), vt = view_of(c, replica * c.N + t, rot);
  // h[(ps' pt'), (ps pt)] = sum over (ps', ps) of E_{ps' ps} (x) h_{ps' ps}, one
  // closed two-column network per non-zero block, plus the norm
  const int d = c.d, dd = d * d;
  std::vector<std::vector<double>> ops;   // pairs (a on s, b on t)
  for (int po = 0; po < d; ++po)
    for (int pi = 0; pi < d; ++pi) {
      std::vector<double> a(dd, 0.0), b(dd, 0.0);
      bool nz = false;
      a[po * d + pi] = 1.0;
      for (int qo = 0; qo < d; ++qo)
        for (int qi = 0; qi < d; ++qi) {
          b[qo * d + qi] = op_host[(po * d + qo) * dd + (pi * d + qi)];
          nz |= (b[qo * d + qi] != 0.0);
        }
      if (nz) {
        ops.push_back(a);
        ops.push_back(b);
      }
    }
  const int nterm = (int)ops.size() / 2;
  double* res = c.arena.alloc(nterm + 1);
  DT LB = left_boundary(c, vs), RB = right_boundary(c, vt);
  double* lslot = c.arena.alloc((size_t)c.chi * c.Db * c.chi);
  const auto m = c.arena.mark();
  for (int k = 0; k <= nterm; ++k) {
    DT Abs = (k < nterm) ? bra_with_op(c, vs.Ab, ops[2 * k].data()) : vs.Ab;
    DT L1 = column(c, LB, vs.T[0], vs.T[2], vs.Ak, Abs, false);   // [t1', R, t3']
    keep(c, L1, lslot);
    DT L1k = make(lslot, L1.dims);
    c.arena.release(m);
    DT Abt = (k < nterm) ? bra_with_op(c, vt.Ab, ops[2 * k + 1].data()) : vt.Ab;
    keep(c, close_lr(c, column(c, L1k, vt.T[0], vt.T[2], vt.Ak, Abt, false), RB), res + k);
    c.arena.release(m);
  }
  const std::vector<double> h = fetch(c, res, nterm + 1);
  double num = 0.0;
  for (int k = 0; k < nterm; ++k) num += h[k];
  return num / h[nterm];
}

size_t observe_arena_elems(long chi, long DK, long DB, long d) {
  // one closed column at a time: the left boundary permuted, X and its
  // permuted copy, Y and its copy, Z and its copy (chi^2 DK^2 DB^2 each, Y
  // times d), T3 permuted, W; plus the boundaries, the kept slot, the
  // operator-carrying bra tensors and the 32-element alignment of each block
  const long c2 = chi * chi, big = c2 * DK * DK * DB * DB, small = c2 * DK * DB;
  return (size_t)(big * (4 + 2 * d) + 16 * small + 8 * DK * DK * DK * DK * d + 64 * 1024);
}

double expect_op(Context& c, const double* rho_dev, const double* op_host, int dim) {
  double* op = c.arena.alloc((size_t)dim * dim + 1);
  CTM_HIP(hipMemcpyAsync(op, op_host, sizeof(double) * dim * dim, hipMemcpyHostToDevice, c.st));
  hipLaunchKernelGGL(k_expect, dim3(1), dim3(64), 0, c.st, rho_dev, op, dim, op + dim * dim);
  CTM_HIP(hipGetLastError());
  return fetch_scalar(c, op + dim * dim);
}

double impurity(Context& c, int site, const double* b_host) {
  c.arena.reset();
  View v = view_of(c, site, 0);
  const long szb = (long)c.DK * c.DK * c.DK * c.DK;
  double* bd = c.arena.alloc(szb);
  CTM_HIP(hipMemcpyAsync(bd, b_host, sizeof(double) * szb, hipMemcpyHostToDevice, c.st));
  DT B = make(bd, {c.DK, c.DK, c.DK, c.DK, 1});
  DT LB = left_boundary(c, v), RB = right_boundary(c, v);
  DT za = close_lr(c, column(c, LB, v.T[0], v.T[2], v.Ak, v.Ab, false), RB);
  DT zb = close_lr(c, column(c, LB, v.T[0], v.T[2], B, v.Ab, false), RB);
  double* r = c.arena.alloc(1);
  hipLaunchKernelGGL(k_ratio, dim3(1), dim3(64), 0, c.st, zb.p, za.p, r);
  CTM_HIP(hipGetLastError());
  return fetch_scalar(c, r);
}

double log_kappa(Context& c) {
  c.arena.reset();
  View v = view_of(c, 0, 0);
  DT LB = left_boundary(c, v), RB = right_boundary(c, v);
  DT z33 = close_lr(c, column(c, LB, v.T[0], v.T[2], v.Ak, v.Ab, false), RB);
  // corners only: trace(C2 C1 C4 C3)
  DT X = tdot(c, v.C[1], {1}, v.C[0], {0});
  X = tdot(c, X, {1}, v.C[3], {0});
  DT zc = tdot(c, X, {0, 1}, v.C[2], {1, 0});
  // two rows, three columns
  DT LB0 = tdot(c, v.C[0], {1}, v.C[3], {0});    // [t1][t3]
  DT RB0 = tdot(c, v.C[1], {0}, v.C[2], {1});    // [t1'][t3']
  DT Y = tdot(c, LB0, {0}, v.T[0], {0});         // [t3][t1'][u]
  Y = tdot(c, Y, {0, 2}, v.T[2], {1, 2});        // [t1'][t3']
  DT z23 = tdot(c, Y, {0, 1}, RB0, {0, 1});
  // three rows, two columns
  DT L = tdot(c, v.C[0], {1}, v.T[3], {1});      // [t][b][l]
  L = tdot(c, L, {1}, v.C[3], {0});              // [t][l][s]
  DT R = tdot(c, v.C[1], {0}, v.T[1], {0});      // [t][e][l]
  R = tdot(c, R, {1}, v.C[2], {1});              // [t][l][s]
  DT z32 = tdot(c, L, {0, 1, 2}, R, {0, 1, 2});
  double* out = c.arena.alloc(1);
  hipLaunchKernelGGL(k_logkappa, dim3(1), dim3(64), 0, c.st, z33.p, zc.p, z23.p, z32.p, out);
  CTM_HIP(hipGetLastError());
  return fetch_scalar(c, out);
}

// ---------------------------------------------------------------------------
// Correlation functions and the transfer-matrix spectrum (Sec. 5.3, Eq. (8)
// and the correlation length of Eq. (9))
// ---------------------------------------------------------------------------
namespace {

// Frame of a walk from `site` along +x (dir 0) or +y (dir 1): the +y walk is
// a +x walk in the frame rotated three quarter turns; (xv, yv) the site's
// position in that frame.
void line_frame(const Context& c, int site, int dir, int& rot, int& xv, int& yv) {
  rot = (dir == 0) ? 0 : 3;
  int x = site % c.Lx, y = site / c.Lx;
  for (int i = 0; i < rot; ++i) { int t = x; x = -y; y = t; }
  xv = x;
  yv = y;
}

// s = x^T y for two device vectors of n elements (one FP64 GEMM), on the device.
void dot_dev(Context& c, const double* x, const double* y, long n, double* s) {
  gemm(c.st, GemmType::F64, 1, 1, (int)n, 1.0, rowmajor(x, n), colmajor(y, n), 0.0, out_colmajor(s, 1), 1, c.ws());
}

}  // namespace

void correlation(Context& c, int site, int dir, const double* opA, const double* opB, int rmax, double* out) {
  const int d = c.d;
  // r = 0: the one-site value of the operator product A B
  std::vector<double> ab((size_t)d * d, 0.0);
  for (int o = 0; o < d; ++o)
    for (int i = 0; i < d; ++i)
      for (int k = 0; k < d; ++k) ab[o * d + i] += opA[o * d + k] * opB[k * d + i];
  out[0] = expect_1site(c, site, ab.data());
  if (rmax <= 0) return;
  c.arena.reset();
  int rot, xv, yv;
  line_frame(c, site, dir, rot, xv, yv);
  CTM_CHECK(view_site(c, rot, xv, yv) == site, -3, "correlation: view bookkeeping");
  const View vs = view_of(c, site, rot);
  const long nb = (long)c.chi * c.Db * c.chi;
  const std::vector<long> bd = {c.chi, c.Db, c.chi};
  double* res = c.arena.alloc(2 * (size_t)rmax);   // (with B, without) per distance
  double* xop = c.arena.alloc(nb);                 // left part with A inserted
  double* xid = c.arena.alloc(nb);                 // left part without operators
  const DT LB = left_boundary(c, vs);
  const auto m0 = c.arena.mark();
  keep(c, column(c, LB, vs.T[0], vs.T[2], vs.Ak, bra_with_op(c, vs.Ab, opA), false), xop);
  c.arena.release(m0);
  keep(c, column(c, LB, vs.T[0], vs.T[2], vs.Ak, vs.Ab, false), xid);
  c.arena.release(m0);
  for (int r = 1; r <= rmax; ++r) {
    const View vj = view_of(c, view_site(c, rot, xv + r, yv), rot);
    const DT Xop = make(xop, bd), Xid = make(xid, bd);
    const DT RB = right_boundary(c, vj);
    keep(c, close_lr(c, column(c, Xop, vj.T[0], vj.T[2], vj.Ak, bra_with_op(c, vj.Ab, opB), false), RB),
         res + 2 * (r - 1));
    const DT nid = column(c, Xid, vj.T[0], vj.T[2], vj.Ak, vj.Ab, false);
    keep(c, close_lr(c, nid, RB), res + 2 * (r - 1) + 1);
    if (r < rmax) {
      // both boundaries move one column on and are divided by the same
      // number (the largest entry of the plain one)
      const DT nop = column(c, Xop, vj.T[0], vj.T[2], vj.Ak, vj.Ab, false);
      normalize_maxabs(c.st, nid.p, nb, c.redscratch.as<double>(), c.badflag.as<int>());
      scale_by_inv(c.st, nop.p, nb, c.redscratch.as<double>() + 1024);
      keep(c, nop, xop);
      keep(c, nid, xid);
    }
    c.arena.release(m0);
  }
  const std::vector<double> h = fetch(c, res, 2 * (size_t)rmax);
  for (int r = 1; r <= rmax; ++r) out[r] = h[2 * (r - 1)] / h[2 * (r - 1) + 1];
  check_bad(c, "ctm_correlation");
}

int transfer_spectrum(Context& c, int dir, int line, int nev, int krylov, double tol, std::complex<double>* lam_out) {
  c.arena.reset();
  const int site = (dir == 0) ? c.Lx * line : line;
  int rot, xv, yv;
  line_frame(c, site, dir, rot, xv, yv);
  const int period = (dir == 0) ? c.Lx : c.Ly;
  const long n = (long)c.chi * c.Db * c.chi;
  const int m = (int)std::min<long>(krylov, n);
  const std::vector<long> bd = {c.chi, c.Db, c.chi};
  std::vector<View> cols(period);
  for (int k = 0; k < period; ++k) cols[k] = view_of(c, view_site(c, rot, xv + k, yv), rot);
  double* V = c.arena.alloc((size_t)n * (m + 1));   // Krylov basis, one vector per row
  double* hd = c.arena.alloc((size_t)m + 8);         // projections of one step
  double* zd = c.arena.alloc((size_t)m + 8);         // restart combination
  const auto mk = c.arena.mark();
  // y = E x: the columns of one period, in order (x and y may not overlap)
  auto matvec = [&](const double* x, double* y) {
    DT X = make(const_cast<double*>(x), bd);
    for (int k = 0; k < period; ++k) X = column(c, X, cols[k].T[0], cols[k].T[2], cols[k].Ak, cols[k].Ab, false);
    keep(c, X, y);
    c.arena.release(mk);
  };
  auto norm_dev = [&](const double* x) {
    dot_dev(c, x, x, n, hd);
    return std::sqrt(std::max(0.0, fetch_scalar(c, hd)));
  };
  // start vector: Philox uniforms on [-1, 1) (fixed key), unit norm
  omega_fill(c.st, V, (int)n, 1, 1, 0x7472616e73666572ull, 0);
  scale(c.st, V, n, 1.0 / norm_dev(V));
  std::vector<std::complex<double>> lam;
  int restarts = 0;
  for (;; ++restarts) {
    std::vector<double> H((size_t)(m + 1) * m, 0.0);
    int me = m;
    double beta = 0.0;
    for (int j = 0; j < m; ++j) {
      double* w = V + (size_t)(j + 1) * n;
      matvec(V + (size_t)j * n, w);
      // classical Gram-Schmidt, applied twice
      for (int pass = 0; pass < 2; ++pass) {
        gemm(c.st, GemmType::F64, j + 1, 1, (int)n, 1.0, rowmajor(V, n), colmajor(w, n), 0.0,
             out_colmajor(hd, j + 1), 1, c.ws());
        gemm(c.st, GemmType::F64, (int)n, 1, j + 1, -1.0, colmajor(V, n), colmajor(hd, j + 1), 1.0,
             out_colmajor(w, n), 1, c.ws());
        const std::vector<double> h = fetch(c, hd, j + 1);
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] += h[i];
      }
      beta = norm_dev(w);
      H[(size_t)(j + 1) * m + j] = beta;
      double hn = 0.0;
      for (int i = 0; i <= j; ++i) hn = std::max(hn, std::fabs(H[(size_t)i * m + j]));
      if (beta <= 1e-14 * std::max(hn, 1e-300)) {   // invariant subspace: the Ritz values are exact
        me = j + 1;
        beta = 0.0;
        break;
      }
      scale(c.st, w, n, 1.0 / beta);
    }
    std::vector<double> Hm((size_t)me * me);
    for (int i = 0; i < me; ++i)
      for (int j = 0; j < me; ++j) Hm[(size_t)i * me + j] = H[(size_t)i * m + j];
    CTM_CHECK(hessenberg_eigenvalues(Hm, me, lam), -4, "transfer spectrum: Hessenberg QR did not converge");
    std::stable_sort(lam.begin(), lam.end(),
                     [](const std::complex<double>& a, const std::complex<double>& b) { return std::abs(a) > std::abs(b); });
    const int want = std::min(nev, me);
    // residual of Ritz pair k: beta |e_m^T y_k| (y_k a unit eigenvector of H_m)
    std::vector<std::vector<std::complex<double>>> Y(want);
    double worst = 0.0;
    for (int k = 0; k < want; ++k) {
      Y[k] = hessenberg_eigenvector(Hm, me, lam[k]);
      worst = std::max(worst, beta * std::abs(Y[k][me - 1]));
    }
    const double scale0 = std::max(std::abs(lam[0]), 1e-300);
    if (beta == 0.0 || worst <= tol * scale0 || restarts >= 40) break;
    // restart from the real combination of the wanted Ritz vectors
    std::vector<double> z(me, 0.0);
    for (int k = 0; k < want; ++k)
      for (int i = 0; i < me; ++i) z[i] += Y[k][i].real() + Y[k][i].imag();
    CTM_HIP(hipMemcpyAsync(zd, z.data(), sizeof(double) * me, hipMemcpyHostToDevice, c.st));
    double* tmp = V + (size_t)m * n;
    gemm(c.st, GemmType::F64, (int)n, 1, me, 1.0, colmajor(V, n), colmajor(zd, me), 0.0, out_colmajor(tmp, n), 1,
         c.ws());
    CTM_HIP(hipMemcpyAsync(V, tmp, sizeof(double) * n, hipMemcpyDeviceToDevice, c.st));
    const double nz = norm_dev(V);
    CTM_CHECK(nz > 0.0, -4, "transfer spectrum: restart vector is zero");
    scale(c.st, V, n, 1.0 / nz);
  }
  for (int k = 0; k < nev; ++k) lam_out[k] = (k < (int)lam.size()) ? lam[k] : 0.0;
  check_bad(c, "ctm_transfer_spectrum");
  return restarts;
}

}  // namespace ctm
