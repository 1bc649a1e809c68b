// Order-0 prolate spheroidal wave function psi_0(c, x) on [-1, 1], float64.
//
// The anti-aliasing function multiplied into every kernel in the image domain
// (Sec. 3.2).  Method: expand psi_0 in even normalised Legendre polynomials;
// the coefficient vector is the eigenvector of the smallest eigenvalue of the
// (symmetric, tridiagonal) matrix of the prolate differential operator
//   -d/dx (1 - x^2) d/dx + c^2 x^2
// in that basis (Bouwkamp 1947; Xiao, Rokhlin & Yarvin 2001).  The small dense
// eigenproblem is solved with cyclic Jacobi rotations.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace pg {
namespace {

// Eigenvector of the smallest eigenvalue of a symmetric matrix a[n*n] (destroyed).
std::vector<double> smallest_eigenvector(std::vector<double>& a, int n) {
  std::vector<double> v(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - s * vkq;
          v[k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  int best = 0;
  for (int i = 1; i < n; ++i)
    if (a[i * n + i] < a[best * n + best]) best = i;
  std::vector<double> out(n);
  for (int k = 0; k < n; ++k) out[k] = v[k * n + best];
  return out;
}

// sum_i coef[i] P_{2i}(x) by the Legendre three-term recurrence.
double even_legendre_series(const std::vector<double>& coef, double x) {
  double p0 = 1.0, p1 = x, sum = coef[0];
  int deg_max = 2 * (static_cast<int>(coef.size()) - 1);
  for (int k = 1; k < deg_max; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
    if ((k + 1) % 2 == 0) sum += coef[(k + 1) / 2] * p2;
  }
  return sum;
}

}  // namespace

std::vector<double> pswf0(double c, const std::vector<double>& x) {
  const int n = static_cast<int>(c) + 40;
  std::vector<double> a(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double k = 2.0 * i;
    a[i * n + i] = k * (k + 1) + c * c * (2 * k * (k + 1) - 1) / ((2 * k + 3) * (2 * k - 1));
    if (i + 1 < n) {
      double e = c * c * (k + 2) * (k + 1) / ((2 * k + 3) * std::sqrt((2 * k + 1) * (2 * k + 5)));
      a[i * n + i + 1] = e;
      a[(i + 1) * n + i] = e;
    }
  }
  std::vector<double> beta = smallest_eigenvector(a, n);
  std::vector<double> coef(n);
  for (int i = 0; i < n; ++i) coef[i] = beta[i] * std::sqrt(2.0 * i + 0.5);  // normalised -> plain basis
  double norm = even_legendre_series(coef, 0.0);
  std::vector<double> out(x.size());
  for (size_t i = 0; i < x.size(); ++i) out[i] = even_legendre_series(coef, x[i]) / norm;
  return out;
}

}  // namespace pg
