// Gauss-Legendre rule on [0,1] by the Golub-Welsch method, in FP64.
//
// The n nodes on [-1,1] are the eigenvalues of the symmetric tridiagonal
// Jacobi matrix of the Legendre recurrence (zero diagonal, off-diagonal
// k / sqrt(4k^2 - 1), k = 1..n-1); the weight of node i is 2 v_{0i}^2, with
// v_i the unit eigenvector.  The eigenproblem is solved with cyclic Jacobi
// rotations, which is simple and accurate for the small n used here.  Nodes
// are mapped to [0,1] by t = (1+x)/2 and 1-t = (1-x)/2 (each computed from x,
// so 1-t keeps full relative precision near t = 1), weights halve.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../qts_internal.h"

namespace qts {

void gauss_legendre(int n, double* t, double* one_minus_t, double* w) {
  if (n < 1 || n > 64) fail(QTS_E_INVALID_ARG, "node count must be in [1, 64]");
  std::vector<double> A((size_t)n * n, 0.0), V((size_t)n * n, 0.0);
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  auto v = [&](int i, int j) -> double& { return V[(size_t)i * n + j]; };
  for (int i = 0; i < n; ++i) v(i, i) = 1.0;
  for (int k = 1; k < n; ++k) {
    const double beta = k / std::sqrt(4.0 * k * k - 1.0);
    a(k - 1, k) = a(k, k - 1) = beta;
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a(p, q) * a(p, q);
    if (off < 1e-60) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        // rotation zeroing a(p,q): tan(2 theta) = 2 a_pq / (a_qq - a_pp)
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) /
                          (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // V <- V J
          const double vkp = v(k, p), vkq = v(k, q);
          v(k, p) = c * vkp - s * vkq;
          v(k, q) = s * vkp + c * vkq;
        }
      }
    }
  }
  std::vector<int> idx((size_t)n);
  for (int i = 0; i < n; ++i) idx[(size_t)i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
  for (int r = 0; r < n; ++r) {
    const int i = idx[(size_t)r];
    double x = a(i, i);
    // the rule is symmetric: x_i = -x_{n-1-i}; enforce it exactly
    if (n % 2 == 1 && r == n / 2) x = 0.0;
    double norm = 0.0;
    for (int k = 0; k < n; ++k) norm += v(k, i) * v(k, i);
    const double v0 = v(0, i);
    t[r] = 0.5 * (1.0 + x);
    one_minus_t[r] = 0.5 * (1.0 - x);
    w[r] = v0 * v0 / norm;  // (2 v0^2) / 2
  }
  // symmetrise: node r and node n-1-r mirror each other
  for (int r = 0; r < n / 2; ++r) {
    const int q = n - 1 - r;
    const double tl = 0.5 * (t[r] + one_minus_t[q]);
    const double th = 0.5 * (one_minus_t[r] + t[q]);
    t[r] = one_minus_t[q] = tl;
    one_minus_t[r] = t[q] = th;
    const double wm = 0.5 * (w[r] + w[q]);
    w[r] = w[q] = wm;
  }
}

}  // namespace qts
