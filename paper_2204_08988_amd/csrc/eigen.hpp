// Symmetric eigendecomposition in float64 on the host (no HIP dependency):
// Householder reduction to tridiagonal form, then implicit symmetric QR steps
// with Wilkinson shifts (Golub & Van Loan, Matrix Computations, 4th ed.,
// Algorithms 8.3.1 and 8.3.3), accumulating every reflection and rotation.
// Cost O(d^3) with a small constant: about 10 d^3 flops.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

namespace dpmm::eig {

// A: row-major d x d symmetric (overwritten).  On return w[j] holds the
// eigenvalues (unsorted) and row j of V (row-major d x d) the unit
// eigenvector of w[j], so that A = V^T diag(w) V.  The accumulated orthogonal
// factor is kept as V = Q^T so that every update runs along contiguous rows.
// Returns false if the QR iteration did not converge.
inline bool sym_eigen(std::vector<double>& A, int d, std::vector<double>& w, std::vector<double>& V) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * d + j]; };
  V.assign((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i) V[(size_t)i * d + i] = 1.0;
  std::vector<double> sr(d);
  std::vector<double> v(d), p(d);
  // 1. tridiagonalise: for column k, reflect rows / columns k+1.. so that
  //    A[k+2.., k] = 0 (H = I - 2 v v^T, |v| = 1; A' = A - 2 (v w^T + w v^T)
  //    with p = A v, w = p - (v^T p) v)
  for (int k = 0; k + 2 < d; ++k) {
    double norm = 0.0;
    for (int i = k + 1; i < d; ++i) norm += a(i, k) * a(i, k);
    norm = std::sqrt(norm);
    if (norm == 0.0) continue;
    const double alpha = a(k + 1, k) > 0.0 ? -norm : norm;
    double vn = 0.0;
    for (int i = k + 1; i < d; ++i) {
      v[i] = a(i, k) - (i == k + 1 ? alpha : 0.0);
      vn += v[i] * v[i];
    }
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < d; ++i) v[i] /= vn;
    double K = 0.0;
    for (int i = k + 1; i < d; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < d; ++j) s += a(i, j) * v[j];
      p[i] = s;
      K += v[i] * s;
    }
    for (int i = k + 1; i < d; ++i) p[i] -= K * v[i];  // p <- w
    for (int i = k + 1; i < d; ++i)
      for (int j = k + 1; j < d; ++j) a(i, j) -= 2.0 * (v[i] * p[j] + p[i] * v[j]);
    a(k + 1, k) = a(k, k + 1) = alpha;
    for (int i = k + 2; i < d; ++i) a(i, k) = a(k, i) = 0.0;
    // Q <- Q H, i.e. V <- H V: V -= 2 v (v^T V) over rows k+1..
    std::fill(sr.begin(), sr.end(), 0.0);
    for (int j = k + 1; j < d; ++j) {
      const double* vr = &V[(size_t)j * d];
      for (int r = 0; r < d; ++r) sr[r] += v[j] * vr[r];
    }
    for (int j = k + 1; j < d; ++j) {
      double* vr = &V[(size_t)j * d];
      const double f = 2.0 * v[j];
      for (int r = 0; r < d; ++r) vr[r] -= f * sr[r];
    }
  }
  // 2. implicit symmetric QR on the tridiagonal T (kept in A's band):
  //    T <- G T G^T and Q <- Q G^T (V <- G V) for Givens rotations G in
  //    planes (k, k+1)
  auto rotate = [&](int k, double c, double s, int lo, int hi) {
    const int j0 = std::max(lo, k - 1), j1 = std::min(hi, k + 2);
    for (int j = j0; j <= j1; ++j) {
      const double x0 = a(k, j), x1 = a(k + 1, j);
      a(k, j) = c * x0 + s * x1;
      a(k + 1, j) = -s * x0 + c * x1;
    }
    for (int j = j0; j <= j1; ++j) {
      const double x0 = a(j, k), x1 = a(j, k + 1);
      a(j, k) = c * x0 + s * x1;
      a(j, k + 1) = -s * x0 + c * x1;
    }
    double* v0 = &V[(size_t)k * d];
    double* v1 = v0 + d;
    for (int r = 0; r < d; ++r) {
      const double x0 = v0[r], x1 = v1[r];
      v0[r] = c * x0 + s * x1;
      v1[r] = -s * x0 + c * x1;
    }
  };
  int hi = d - 1, iters = 0;
  while (hi > 0) {
    if (++iters > 60 * d + 60) return false;
    for (int i = 0; i < hi; ++i)
      if (std::fabs(a(i + 1, i)) <= 1e-16 * (std::fabs(a(i, i)) + std::fabs(a(i + 1, i + 1))) ||
          std::fabs(a(i + 1, i)) < 1e-300)
        a(i + 1, i) = a(i, i + 1) = 0.0;
    while (hi > 0 && a(hi, hi - 1) == 0.0) --hi;
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && a(lo, lo - 1) != 0.0) --lo;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer T[hi][hi]
    const double dd = 0.5 * (a(hi - 1, hi - 1) - a(hi, hi));
    const double b = a(hi, hi - 1);
    const double mu = a(hi, hi) - b * b / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, b));
    double x = a(lo, lo) - mu, z = a(lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : z / r;
      rotate(k, c, s, lo, hi);
      if (k + 1 < hi) {
        x = a(k + 1, k);  // chase the bulge at (k + 2, k)
        z = a(k + 2, k);
      }
    }
  }
  w.resize(d);
  for (int i = 0; i < d; ++i) w[i] = a(i, i);
  return true;
}

}  // namespace dpmm::eig
