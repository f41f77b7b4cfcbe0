// Host eigen-solver for small upper Hessenberg matrices (see hessenberg.hpp).
#include "hessenberg.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>

namespace ctm {
namespace {

// Householder reflector for a vector of length 2 or 3: I - beta v v^T maps x
// to a multiple of e_1; v[0] = 1.  beta = 0 when x is already such a multiple.
void house(const double* x, int len, double* v, double& beta) {
  double sigma = 0.0;
  for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
  v[0] = 1.0;
  for (int i = 1; i < len; ++i) v[i] = x[i];
  if (sigma == 0.0) {
    beta = 0.0;
    return;
  }
  const double mu = std::sqrt(x[0] * x[0] + sigma);
  const double v0 = (x[0] <= 0.0) ? x[0] - mu : -sigma / (x[0] + mu);
  beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
  for (int i = 1; i < len; ++i) v[i] /= v0;
}

// Eigenvalues of the 2 x 2 block [[a, b], [c, d]].
void eig2(double a, double b, double c, double d, std::complex<double>& l1, std::complex<double>& l2) {
  const double p = 0.5 * (a - d), disc = p * p + b * c, mid = 0.5 * (a + d);
  if (disc >= 0.0) {
    const double r = std::sqrt(disc);
    // the root of larger modulus first, the other from the determinant
    const double big = mid + (mid >= 0.0 ? r : -r);
    const double det = a * d - b * c;
    l1 = big;
    l2 = (big != 0.0) ? det / big : mid - (mid >= 0.0 ? r : -r);
  } else {
    const double r = std::sqrt(-disc);
    l1 = std::complex<double>(mid, r);
    l2 = std::complex<double>(mid, -r);
  }
}

}  // namespace

bool hessenberg_eigenvalues(std::vector<double> H, int n, std::vector<std::complex<double>>& lam) {
  lam.assign(n, 0.0);
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
  for (int i = 0; i < n; ++i)
    for (int j = 0; j + 1 < i; ++j) h(i, j) = 0.0;
  double norm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = std::max(0, i - 1); j < n; ++j) norm = std::max(norm, std::fabs(h(i, j)));
  int hi = n - 1, its = 0, total = 0;
  while (hi >= 0) {
    // negligible subdiagonal entries inside the active part become zero
    for (int i = hi; i >= 1; --i) {
      double s = std::fabs(h(i - 1, i - 1)) + std::fabs(h(i, i));
      if (s == 0.0) s = norm;
      if (std::fabs(h(i, i - 1)) <= DBL_EPSILON * s) h(i, i - 1) = 0.0;
    }
    int lo = hi;
    while (lo > 0 && h(lo, lo - 1) != 0.0) --lo;
    if (lo == hi) {                       // a 1 x 1 block has split off
      lam[hi] = h(hi, hi);
      hi -= 1;
      its = 0;
      continue;
    }
    if (lo == hi - 1) {                   // a 2 x 2 block has split off
      eig2(h(hi - 1, hi - 1), h(hi - 1, hi), h(hi, hi - 1), h(hi, hi), lam[hi - 1], lam[hi]);
      hi -= 2;
      its = 0;
      continue;
    }
    if (++total > 40 * n) return false;
    ++its;
    // shifts: the eigenvalues of the trailing 2 x 2 block (through their sum
    // s and product t), or an exceptional pair every tenth step
    double s, t;
    if (its % 10 == 0) {
      const double e = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
      s = 1.5 * e + h(hi, hi);
      t = e * e;
    } else {
      s = h(hi - 1, hi - 1) + h(hi, hi);
      t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
    }
    // first column of (H - l1)(H - l2) restricted to the window lo..hi
    double x = h(lo, lo) * h(lo, lo) + h(lo, lo + 1) * h(lo + 1, lo) - s * h(lo, lo) + t;
    double y = h(lo + 1, lo) * (h(lo, lo) + h(lo + 1, lo + 1) - s);
    double z = h(lo + 1, lo) * h(lo + 2, lo + 1);
    // chase the bulge down the window with 3-vector reflectors (the
    // similarity acts on the window only: its eigenvalues are all we need)
    for (int k = lo; k <= hi - 2; ++k) {
      const double xv[3] = {x, y, z};
      double v[3], beta;
      house(xv, 3, v, beta);
      if (beta != 0.0) {
        const int c0 = std::max(lo, k - 1);
        for (int j = c0; j <= hi; ++j) {
          const double w = beta * (v[0] * h(k, j) + v[1] * h(k + 1, j) + v[2] * h(k + 2, j));
          h(k, j) -= w * v[0];
          h(k + 1, j) -= w * v[1];
          h(k + 2, j) -= w * v[2];
        }
        const int r1 = std::min(k + 3, hi);
        for (int i = lo; i <= r1; ++i) {
          const double w = beta * (h(i, k) * v[0] + h(i, k + 1) * v[1] + h(i, k + 2) * v[2]);
          h(i, k) -= w * v[0];
          h(i, k + 1) -= w * v[1];
          h(i, k + 2) -= w * v[2];
        }
      }
      x = h(k + 1, k);
      y = h(k + 2, k);
      if (k < hi - 2) z = h(k + 3, k);
    }
    const double xv[2] = {x, y};
    double v[3], beta;
    house(xv, 2, v, beta);
    if (beta != 0.0) {
      for (int j = hi - 2; j <= hi; ++j) {
        const double w = beta * (v[0] * h(hi - 1, j) + v[1] * h(hi, j));
        h(hi - 1, j) -= w * v[0];
        h(hi, j) -= w * v[1];
      }
      for (int i = lo; i <= hi; ++i) {
        const double w = beta * (h(i, hi - 1) * v[0] + h(i, hi) * v[1]);
        h(i, hi - 1) -= w * v[0];
        h(i, hi) -= w * v[1];
      }
    }
    // the reflectors leave round-off below the subdiagonal of the window
    for (int i = lo + 2; i <= hi; ++i)
      for (int j = lo; j < i - 1; ++j) h(i, j) = 0.0;
  }
  return true;
}

std::vector<std::complex<double>> hessenberg_eigenvector(const std::vector<double>& H, int n,
                                                        std::complex<double> lam) {
  using cd = std::complex<double>;
  double norm = 0.0;
  for (double v : H) norm = std::max(norm, std::fabs(v));
  const double tiny = std::max(norm, 1e-300) * DBL_EPSILON;
  // LU of H - lam I with partial pivoting (row-major, complex)
  std::vector<cd> A((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = (j + 1 >= i ? H[(size_t)i * n + j] : 0.0) - (i == j ? lam : 0.0);
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A[(size_t)i * n + k]) > std::abs(A[(size_t)p * n + k])) p = i;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
    if (std::abs(A[(size_t)k * n + k]) < tiny) A[(size_t)k * n + k] = tiny;
    const cd d = A[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      const cd f = A[(size_t)i * n + k] / d;
      A[(size_t)i * n + k] = f;
      if (f != cd(0.0))
        for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
    }
  }
  std::vector<cd> x(n, cd(1.0));
  for (int step = 0; step < 2; ++step) {
    for (int k = 0; k < n; ++k) std::swap(x[k], x[piv[k]]);
    for (int i = 1; i < n; ++i)
      for (int j = 0; j < i; ++j) x[i] -= A[(size_t)i * n + j] * x[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) x[i] -= A[(size_t)i * n + j] * x[j];
      x[i] /= A[(size_t)i * n + i];
    }
    double nrm = 0.0;
    for (const cd& v : x) nrm += std::norm(v);
    nrm = std::sqrt(nrm);
    for (cd& v : x) v /= nrm;
  }
  return x;
}

}  // namespace ctm
