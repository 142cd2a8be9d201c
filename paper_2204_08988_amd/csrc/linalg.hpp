// Workgroup-parallel float64 dense kernels for one small d x d matrix held in
// LDS (or global scratch), row-major.  All are right-looking: at step j the
// whole workgroup updates the trailing part in parallel, so every step costs a
// few barriers and independent LDS accesses instead of a serial dot product.
#pragma once
#include "common.hpp"

namespace dpmm {

// In-place lower Cholesky a = L L^T; the strict upper triangle is zeroed.
// Returns false (on every thread) if a pivot is not positive and finite.
__device__ inline bool wg_cholesky(double* a, int d, int* flag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) *flag = 1;
  __syncthreads();
  for (int j = 0; j < d; ++j) {
    if (tid == 0) {
      double s = a[j * d + j];
      if (!(s > 0.0) || !isfinite(s)) {
        *flag = 0;
        s = 1.0;
      }
      a[j * d + j] = sqrt(s);
    }
    __syncthreads();
    const double inv = 1.0 / a[j * d + j];
    for (int i = j + 1 + tid; i < d; i += nt) a[i * d + j] *= inv;
    __syncthreads();
    // trailing update of the lower triangle: a_ik -= a_ij a_kj, j < k <= i
    const int m = d - j - 1;
    for (int idx = tid; idx < m * m; idx += nt) {
      const int i = j + 1 + idx / m, k = j + 1 + idx % m;
      if (k <= i) a[i * d + k] -= a[i * d + j] * a[k * d + j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < d * d; idx += nt) {
    const int i = idx / d, j = idx % d;
    if (j > i) a[idx] = 0.0;
  }
  __syncthreads();
  const bool ok = *flag != 0;
  __syncthreads();
  return ok;
}

// W = G^-1 for lower-triangular G (W lower triangular), W must not alias G.
__device__ inline void wg_lower_inverse(const double* G, double* W, int d) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < d * d; idx += nt) W[idx] = (idx / d == idx % d) ? 1.0 : 0.0;
  __syncthreads();
  // forward elimination on [G | I] one row at a time: row j of W is final
  // after dividing by G_jj; it is then eliminated from the rows below.
  for (int j = 0; j < d; ++j) {
    const double inv = 1.0 / G[j * d + j];
    for (int c = tid; c <= j; c += nt) W[j * d + c] *= inv;
    __syncthreads();
    const int m = d - j - 1;
    for (int idx = tid; idx < m * (j + 1); idx += nt) {
      const int i = j + 1 + idx / (j + 1), c = idx % (j + 1);
      W[i * d + c] -= G[i * d + j] * W[j * d + c];
    }
    __syncthreads();
  }
}

// F = B A^-T for lower-triangular A, in place on F (F holds B on entry):
// column j of F is final after dividing by A_jj, then removed from the later
// columns, F[:, q] -= F[:, j] A[q][j] for q > j.
__device__ inline void wg_right_solve_lower_t(double* F, const double* A, int d) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = 0; j < d; ++j) {
    const double inv = 1.0 / A[j * d + j];
    for (int r = tid; r < d; r += nt) F[r * d + j] *= inv;
    __syncthreads();
    const int m = d - j - 1;
    for (int idx = tid; idx < d * m; idx += nt) {
      const int r = idx / m, q = j + 1 + idx % m;
      F[r * d + q] -= F[r * d + j] * A[q * d + j];
    }
    __syncthreads();
  }
}

}  // namespace dpmm
